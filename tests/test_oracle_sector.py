"""Pins of the oracle's particle-number / S_z restricted state vector.

References not computed by the code under test: the full-space oracle
(itself pinned against dense matrices), the closed-form Hartree-Fock energy,
the counting formula C(n, N_alpha) C(n, N_beta), exact diagonalization in the
sector, and second quantization on bit strings."""
from math import comb

import numpy as np
import pytest

import qf_inputs as qi
from oracle import ansatz as an, dense, hamiltonian as ham, sector, statevec as sv


@pytest.mark.parametrize("n_orb,na,nb", [(4, 2, 2), (5, 3, 2), (6, 3, 3)])
def test_sector_size_order_and_round_trip(n_orb, na, nb):
    dets = sector.determinants(n_orb, na, nb)
    assert len(dets) == comb(n_orb, na) * comb(n_orb, nb) == len(set(dets.tolist()))
    for y in dets:
        a = sum(((int(y) >> (2 * j)) & 1) << j for j in range(n_orb))
        b = sum(((int(y) >> (2 * j + 1)) & 1) << j for j in range(n_orb))
        assert bin(a).count("1") == na and bin(b).count("1") == nb
    n = 2 * n_orb
    v = qi.random_state(n, 7)
    assert np.array_equal(sector.restrict(sector.embed(sector.restrict(v, n_orb, na, nb), n_orb, na, nb),
                                          n_orb, na, nb), sector.restrict(v, n_orb, na, nb))


@pytest.mark.parametrize("n_orb,n_elec,seed", [(4, 4, 1008), (5, 3, 61), (6, 6, 62)])
def test_sector_ansatz_and_energy_equal_full_space(n_orb, n_elec, seed):
    n = 2 * n_orb
    na, nb = (n_elec + 1) // 2, n_elec // 2
    h, g = qi.integrals(n_orb, n_elec, seed)
    hx, hz, hc, goff = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    excs, ax, az, ac, aoff, _ = an.build(n_orb, n_elec)
    t = qi.amplitudes(len(excs), seed, 0.3)
    occ = an.reference_mask(n_elec)
    full = sv.apply_product(sv.prepare(n, occ), n, ax, az, an.angles(ac, aoff, t))
    # the full-space state never leaves the sector
    assert np.linalg.norm(full) == pytest.approx(np.linalg.norm(sector.restrict(full, n_orb, na, nb)), abs=1e-13)
    ps = sector.apply_excitations(sector.prepare(n_orb, na, nb, occ), n_orb, na, nb, excs, t)
    assert np.allclose(ps, sector.restrict(full, n_orb, na, nb), atol=1e-13)
    e = sector.energy(ps, n_orb, na, nb, hx, hz, hc, goff)
    assert e == pytest.approx(sv.energy(full, n, hx, hz, hc), abs=1e-12)


def test_sector_hf_energy_and_ground_state_bound():
    n_orb, n_elec = 4, 4
    h, g = qi.integrals(n_orb, n_elec, 1008)
    hx, hz, hc, goff = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    ps = sector.prepare(n_orb, 2, 2, 15)
    e_hf = 2 * sum(h[i, i] for i in range(2)) + sum(2 * g[i, i, j, j] - g[i, j, j, i] for i in range(2)
                                                    for j in range(2))
    assert sector.energy(ps, n_orb, 2, 2, hx, hz, hc, goff) == pytest.approx(e_hf, abs=1e-12)
    hd = dense.fermion_matrix(list(ham.fermion_hamiltonian_terms(h, g)), 8)
    e0 = dense.ground_energy_in_sector(hd, 8, 4, 0)
    excs = an.excitations(8, 4)
    for seed in range(3):
        t = qi.amplitudes(len(excs), 300 + seed, 1.0)
        ps = sector.apply_excitations(sector.prepare(n_orb, 2, 2, 15), n_orb, 2, 2, excs, t)
        assert np.vdot(ps, ps).real == pytest.approx(1.0, abs=1e-12)
        assert sector.energy(ps, n_orb, 2, 2, hx, hz, hc, goff) >= e0 - 1e-12


def test_sector_rotation_signs_match_second_quantization():
    # one excitation from a random sector state: compare with the dense
    # exp(t (tau - tau^dagger)) built on bit strings, restricted to the sector
    from scipy.linalg import expm
    n_orb, na, nb = 4, 2, 2
    psi_full = sector.embed(sector.restrict(qi.random_state(8, 9), 4, 2, 2), 4, 2, 2)
    psi_full /= np.linalg.norm(psi_full)
    for cre, ann in an.excitations(8, 4)[:10]:
        K = dense.fermion_matrix([(1.0, cre, ann), (-1.0, tuple(reversed(ann)), tuple(reversed(cre)))], 8)
        want = sector.restrict(expm(0.7 * K) @ psi_full, n_orb, na, nb)
        got = sector.apply_excitations(sector.restrict(psi_full, n_orb, na, nb), n_orb, na, nb, [(cre, ann)], [0.7])
        assert np.allclose(got, want, atol=1e-13)
