"""Python face of the C ABI: the same calls, torch tensors for device memory.

Each function checks the status code of the C call and raises QFError on
failure.  States are complex128 CUDA(ROCm) tensors of length 2**n_qubits.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import TERM_DTYPE, check, lib, ptr, stream_handle

KINDS = {"hamiltonian": _lib.QF_HAMILTONIAN, "uccsd": _lib.QF_UCCSD, "uccd": _lib.QF_UCCD,
         "uccd_top": _lib.QF_UCCD_TOP, "puccd": _lib.QF_PUCCD, "gsd_pool": _lib.QF_GSD_POOL}


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def build_paulis(kind: str, n_orb: int, n_elec: int, h=None, g=None, e_core: float = 0.0,
                 t_rank=None, top_k: int = 0):
    """qf_build_paulis: returns (terms[TERM_DTYPE], off[int64], kept[int64] or None)."""
    k = KINDS[kind]
    h, g, t_rank = _f64(h), _f64(g), _f64(t_rank)
    n_out, n_off = ctypes.c_int64(), ctypes.c_int64()
    check(lib.qf_build_paulis(k, n_orb, n_elec, ptr(h), ptr(g), e_core, ptr(t_rank), int(top_k),
                              None, 0, ctypes.byref(n_out), None, 0, ctypes.byref(n_off), None),
          "qf_build_paulis(size)")
    terms = np.zeros(n_out.value, dtype=TERM_DTYPE)
    off = np.zeros(n_off.value, dtype=np.int64)
    kept = np.zeros(max(n_off.value - 1, 0), dtype=np.int64) if k != _lib.QF_HAMILTONIAN else None
    check(lib.qf_build_paulis(k, n_orb, n_elec, ptr(h), ptr(g), e_core, ptr(t_rank), int(top_k),
                              ptr(terms), len(terms), ctypes.byref(n_out), ptr(off), len(off),
                              ctypes.byref(n_off), ptr(kept)), "qf_build_paulis")
    return terms, off, kept


def ansatz_angles(A: np.ndarray, exc_off: np.ndarray, t) -> np.ndarray:
    t = _f64(t)
    theta = np.zeros(len(A), dtype=np.float64)
    exc_off = np.ascontiguousarray(exc_off, dtype=np.int64)
    check(lib.qf_ansatz_angles(ptr(A), ptr(exc_off), len(exc_off) - 1, ptr(t), ptr(theta)), "qf_ansatz_angles")
    return theta


def grad_t(A: np.ndarray, exc_off: np.ndarray, dtheta) -> np.ndarray:
    dtheta = _f64(dtheta)
    exc_off = np.ascontiguousarray(exc_off, dtype=np.int64)
    out = np.zeros(len(exc_off) - 1, dtype=np.float64)
    check(lib.qf_grad_t(ptr(A), ptr(exc_off), len(exc_off) - 1, ptr(dtheta), ptr(out)), "qf_grad_t")
    return out


def prepare_state(psi, n_qubits: int, occ_mask: int, stream=None) -> None:
    check(lib.qf_prepare_state(ptr(psi), n_qubits, occ_mask, stream_handle(stream)), "qf_prepare_state")


def apply_pauli_exp(psi, n_qubits: int, terms: np.ndarray, theta, inverse: bool = False, stream=None) -> None:
    theta = _f64(theta)
    check(lib.qf_apply_pauli_exp(ptr(psi), n_qubits, ptr(terms), ptr(theta), len(terms), int(inverse),
                                 stream_handle(stream)), "qf_apply_pauli_exp")


def energy(psi, n_qubits: int, H: np.ndarray, group_off: np.ndarray, stream=None) -> float:
    group_off = np.ascontiguousarray(group_off, dtype=np.int64)
    e = ctypes.c_double()
    check(lib.qf_energy(ptr(psi), n_qubits, ptr(H), ptr(group_off), len(group_off) - 1, ctypes.byref(e),
                        stream_handle(stream)), "qf_energy")
    return e.value


def energy_grad(n_qubits: int, occ_mask: int, A: np.ndarray, theta, H: np.ndarray, group_off: np.ndarray,
                workspace=None, stream=None):
    """Returns (E, dE/dtheta).  workspace: complex128 tensor of 2 * 2**n (allocated if None)."""
    import torch
    theta = _f64(theta)
    group_off = np.ascontiguousarray(group_off, dtype=np.int64)
    if workspace is None:
        workspace = torch.empty(2 << n_qubits, dtype=torch.complex128, device="cuda")
    e = ctypes.c_double()
    g = np.zeros(len(A), dtype=np.float64)
    check(lib.qf_energy_grad(n_qubits, occ_mask, ptr(A), ptr(theta), len(A), ptr(H), ptr(group_off),
                             len(group_off) - 1, ptr(workspace), ctypes.byref(e), ptr(g),
                             stream_handle(stream)), "qf_energy_grad")
    return e.value, g


def energy_static(psi, n_qubits: int, H: np.ndarray, group_off: np.ndarray, stream=None) -> float:
    """qf_energy_static: qf_energy with no device allocation (the library's
    static scratch holds the tables); calls on one GPU must not overlap."""
    group_off = np.ascontiguousarray(group_off, dtype=np.int64)
    e = ctypes.c_double()
    check(lib.qf_energy_static(ptr(psi), n_qubits, ptr(H), ptr(group_off), len(group_off) - 1, ctypes.byref(e),
                               stream_handle(stream)), "qf_energy_static")
    return e.value


def pool_grad(n_qubits: int, occ_mask: int, A: np.ndarray, theta, H: np.ndarray, group_off: np.ndarray,
              pool: np.ndarray, pool_off: np.ndarray, workspace=None, stream=None):
    """qf_pool_grad: (E, g) with g_nu = <Psi|[H, kappa_nu]|Psi> for the pool
    members (ADAPT-VQE, Sec. 3.2) at Psi = U(theta)|occ_mask>."""
    import torch
    theta = _f64(theta)
    group_off = np.ascontiguousarray(group_off, dtype=np.int64)
    pool_off = np.ascontiguousarray(pool_off, dtype=np.int64)
    if workspace is None:
        workspace = torch.empty(2 << n_qubits, dtype=torch.complex128, device="cuda")
    e = ctypes.c_double()
    g = np.zeros(len(pool_off) - 1, dtype=np.float64)
    check(lib.qf_pool_grad(n_qubits, occ_mask, ptr(A), ptr(theta), 0 if A is None else len(A), ptr(H),
                           ptr(group_off), len(group_off) - 1, ptr(pool), ptr(pool_off), len(pool_off) - 1,
                           ptr(workspace), ctypes.byref(e), ptr(g), stream_handle(stream)), "qf_pool_grad")
    return e.value, g


def excited_determinants(kind: str, n_orb: int, n_elec: int, t_rank=None, top_k: int = 0):
    """qf_excited_determinants: (det[uint64], sign[int32]) with
    tau_mu |ref> = sign_mu |det_mu> per excitation of the ansatz kind."""
    t_rank = _f64(t_rank)
    n = ctypes.c_int64()
    check(lib.qf_excited_determinants(KINDS[kind], n_orb, n_elec, ptr(t_rank), int(top_k), None, None, 0,
                                      ctypes.byref(n)), "qf_excited_determinants(size)")
    det = np.zeros(n.value, dtype=np.uint64)
    sign = np.zeros(n.value, dtype=np.int32)
    check(lib.qf_excited_determinants(KINDS[kind], n_orb, n_elec, ptr(t_rank), int(top_k), ptr(det), ptr(sign),
                                      n.value, ctypes.byref(n)), "qf_excited_determinants")
    return det, sign


def mp_denominators(kind: str, n_orb: int, n_elec: int, h, g, t_rank=None, top_k: int = 0) -> np.ndarray:
    """qf_mp_denominators: Delta_mu of Eq. (fixed_point) per excitation."""
    h, g, t_rank = _f64(h), _f64(g), _f64(t_rank)
    n = ctypes.c_int64()
    check(lib.qf_mp_denominators(KINDS[kind], n_orb, n_elec, ptr(h), ptr(g), ptr(t_rank), int(top_k), None, 0,
                                 ctypes.byref(n)), "qf_mp_denominators(size)")
    out = np.zeros(n.value, dtype=np.float64)
    check(lib.qf_mp_denominators(KINDS[kind], n_orb, n_elec, ptr(h), ptr(g), ptr(t_rank), int(top_k), ptr(out),
                                 n.value, ctypes.byref(n)), "qf_mp_denominators")
    return out


def pqe_residuals(n_qubits: int, occ_mask: int, A: np.ndarray, theta, H: np.ndarray, group_off: np.ndarray,
                  det: np.ndarray, sign: np.ndarray, workspace=None, stream=None):
    """qf_pqe_residuals: (E, r) with r_mu = <Phi_mu|U^dagger H U|Phi_0> (Sec. 3.3)."""
    import torch
    theta = _f64(theta)
    group_off = np.ascontiguousarray(group_off, dtype=np.int64)
    det = np.ascontiguousarray(det, dtype=np.uint64)
    sign = np.ascontiguousarray(sign, dtype=np.int32)
    if workspace is None:
        workspace = torch.empty(2 << n_qubits, dtype=torch.complex128, device="cuda")
    e = ctypes.c_double()
    r = np.zeros(len(det), dtype=np.float64)
    check(lib.qf_pqe_residuals(n_qubits, occ_mask, ptr(A), ptr(theta), len(A), ptr(H), ptr(group_off),
                               len(group_off) - 1, ptr(det), ptr(sign), len(det), ptr(workspace), ctypes.byref(e),
                               ptr(r), stream_handle(stream)), "qf_pqe_residuals")
    return e.value, r


def excitations(kind: str, n_orb: int, n_elec: int, t_rank=None, top_k: int = 0) -> np.ndarray:
    """qf_excitations: int32 [n_par, 4] rows (c0, c1, a0, a1) of
    tau = a+_c0 a+_c1 a_a0 a_a1 (-1 where a single has no second operator)."""
    t_rank = _f64(t_rank)
    n = ctypes.c_int64()
    check(lib.qf_excitations(KINDS[kind], n_orb, n_elec, ptr(t_rank), int(top_k), None, 0, ctypes.byref(n)),
          "qf_excitations(size)")
    ops = np.zeros((n.value, 4), dtype=np.int32)
    check(lib.qf_excitations(KINDS[kind], n_orb, n_elec, ptr(t_rank), int(top_k), ptr(ops), n.value,
                             ctypes.byref(n)), "qf_excitations")
    return ops


class Sector:
    """qf_sector_*: the (N_alpha, N_beta) restricted state vector.  States are
    complex128 tensors of `dim` entries (alpha-string rank major)."""

    def __init__(self, n_orb: int, n_alpha: int, n_beta: int, exc=None, H=None, group_off=None):
        self.n_orb = n_orb
        self._exc = None if exc is None else np.ascontiguousarray(exc, dtype=np.int32)
        self._goff = None if group_off is None else np.ascontiguousarray(group_off, dtype=np.int64)
        self._H = H
        ne = 0 if self._exc is None else len(self._exc)
        G = 0 if self._goff is None else len(self._goff) - 1
        h = ctypes.c_void_p()
        check(lib.qf_sector_create(n_orb, n_alpha, n_beta, ptr(self._exc), ne, ptr(H), ptr(self._goff), G,
                                   ctypes.byref(h)), "qf_sector_create")
        self._h = h
        d, da, db, g = (ctypes.c_int64() for _ in range(4))
        check(lib.qf_sector_info(h, ctypes.byref(d), ctypes.byref(da), ctypes.byref(db), ctypes.byref(g)),
              "qf_sector_info")
        self.dim, self.d_alpha, self.d_beta, self.groups = d.value, da.value, db.value, g.value

    def close(self, _destroy=lib.qf_sector_destroy):
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def prepare(self, psi, occ_mask: int, stream=None) -> None:
        check(lib.qf_sector_prepare(self._h, ptr(psi), int(occ_mask), stream_handle(stream)), "qf_sector_prepare")

    def apply(self, psi, t, inverse: bool = False, stream=None) -> None:
        t = _f64(t)
        check(lib.qf_sector_apply(self._h, ptr(psi), ptr(t), int(inverse), stream_handle(stream)), "qf_sector_apply")

    def energy(self, psi, stream=None) -> float:
        e = ctypes.c_double()
        check(lib.qf_sector_energy(self._h, ptr(psi), ctypes.byref(e), stream_handle(stream)), "qf_sector_energy")
        return e.value

    def energy_grad(self, occ_mask: int, t, workspace=None, stream=None):
        """qf_sector_energy_grad: (E, dE/dt) with one derivative per
        excitation.  workspace: complex128 tensor of 2 * dim (allocated if None)."""
        import torch
        t = _f64(t)
        if workspace is None:
            workspace = torch.empty(2 * self.dim, dtype=torch.complex128, device="cuda")
        e = ctypes.c_double()
        g = np.zeros(0 if self._exc is None else len(self._exc), dtype=np.float64)
        check(lib.qf_sector_energy_grad(self._h, int(occ_mask), ptr(t), ptr(workspace), ctypes.byref(e), ptr(g),
                                        stream_handle(stream)), "qf_sector_energy_grad")
        return e.value, g


class PoolPlan:
    """qf_plan_create_pool: device tables of an ADAPT operator pool."""

    def __init__(self, n_qubits: int, pool: np.ndarray, pool_off: np.ndarray):
        self.n = n_qubits
        self.pool_off = np.ascontiguousarray(pool_off, dtype=np.int64)
        self.n_pool = len(self.pool_off) - 1
        self._pool = pool
        h = ctypes.c_void_p()
        check(lib.qf_plan_create_pool(n_qubits, ptr(pool), ptr(self.pool_off), self.n_pool, ctypes.byref(h)),
              "qf_plan_create_pool")
        self._h = h

    def apply_info(self) -> dict:
        bb = ctypes.c_int()
        r = ctypes.c_int64()
        ps = ctypes.c_int64()
        check(lib.qf_plan_apply_info(self._h, ctypes.byref(bb), ctypes.byref(r), ctypes.byref(ps)),
              "qf_plan_apply_info")
        return {"block_bits": bb.value, "runs": r.value, "passes": ps.value}

    def grad_info(self) -> dict:
        """Read-only passes of the pool sweep."""
        b = ctypes.c_int64()
        check(lib.qf_plan_grad_info(self._h, None, ctypes.byref(b)), "qf_plan_grad_info")
        return {"sweep_passes": b.value}

    def close(self, _destroy=lib.qf_plan_destroy):
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


_PLAN_TILES = None


def _plan_tiles() -> dict:
    global _PLAN_TILES
    if _PLAN_TILES is None:
        from .autotune import device_arch, load_plan_table
        _PLAN_TILES = load_plan_table(device_arch())
    return _PLAN_TILES


class Plan:
    """qf_plan_*: device-resident ansatz and Hamiltonian tables for repeated calls.

    tuned: apply the autotuned tiles for this qubit count (blocked-apply
    sub-cube bits, energy tile bits) from the committed table when it was
    measured on this device architecture; False keeps the library defaults.
    """

    def __init__(self, n_qubits: int, A: np.ndarray | None = None, H: np.ndarray | None = None,
                 group_off: np.ndarray | None = None, tuned: bool = True, arena=None, stream=None):
        """arena: (device address, bytes) of a caller buffer that receives the
        plan's device tables (qf_plan_create_arena; size from arena_bytes());
        the plan then allocates and frees no device memory."""
        self.n = n_qubits
        self.K = 0 if A is None else len(A)
        self._A = A
        self._H = H
        self._goff = None if group_off is None else np.ascontiguousarray(group_off, dtype=np.int64)
        G = 0 if self._goff is None else len(self._goff) - 1
        h = ctypes.c_void_p()
        if arena is not None:
            bb, et = self._tiles(n_qubits, self.K, G, tuned)
            need = ctypes.c_int64()
            check(lib.qf_plan_create_arena(n_qubits, ptr(A), self.K, ptr(H), ptr(self._goff), G, bb, et,
                                           ctypes.c_void_p(int(arena[0])), int(arena[1]), ctypes.byref(need),
                                           stream_handle(stream), ctypes.byref(h)), "qf_plan_create_arena")
            self._h = h
            return
        check(lib.qf_plan_create(n_qubits, ptr(A), self.K, ptr(H), ptr(self._goff), G, ctypes.byref(h)),
              "qf_plan_create")
        self._h = h
        if tuned:
            # the autotuned tiles for this qubit count, when the committed
            # table matches this device (else the library's defaults)
            t = _plan_tiles().get(int(n_qubits))
            if t:
                if self.K and t.get("block_bits"):
                    self.set_block_bits(int(t["block_bits"]))
                if G and t.get("energy_tile") and n_qubits > int(t["energy_tile"]):
                    self.set_energy_tile(int(t["energy_tile"]), True)

    @staticmethod
    def _tiles(n: int, K: int, G: int, tuned: bool):
        """(block_bits, energy_tile) for an arena plan: the autotuned values
        for this qubit count when the table matches the device, else -1
        (library defaults)."""
        t = _plan_tiles().get(int(n)) if tuned else None
        bb = int(t["block_bits"]) if (t and K and t.get("block_bits")) else -1
        et = int(t["energy_tile"]) if (t and G and t.get("energy_tile") and n > int(t["energy_tile"])) else -1
        return bb, et

    @staticmethod
    def arena_bytes(n_qubits: int, A=None, H=None, group_off=None, tuned: bool = True) -> int:
        """Device bytes an arena plan of these tables needs."""
        K = 0 if A is None else len(A)
        goff = None if group_off is None else np.ascontiguousarray(group_off, dtype=np.int64)
        G = 0 if goff is None else len(goff) - 1
        bb, et = Plan._tiles(n_qubits, K, G, tuned)
        need = ctypes.c_int64()
        check(lib.qf_plan_create_arena(n_qubits, ptr(A), K, ptr(H), ptr(goff), G, bb, et, None, 0,
                                       ctypes.byref(need), None, None), "qf_plan_create_arena(size)")
        return need.value

    def close(self, _destroy=lib.qf_plan_destroy):
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_energy_tile(self, tile_bits: int, merged: bool = True) -> None:
        """0: one pass per flip-mask group; 10-12: tiled passes per class
        (merged: strings sharing their low Z bits evaluated once per tile)."""
        check(lib.qf_plan_set_energy_tile(self._h, int(tile_bits), int(merged)), "qf_plan_set_energy_tile")

    def info(self) -> dict:
        tb = ctypes.c_int()
        cl = ctypes.c_int64()
        ps = ctypes.c_int64()
        check(lib.qf_plan_info(self._h, ctypes.byref(tb), ctypes.byref(cl), ctypes.byref(ps)), "qf_plan_info")
        return {"tile_bits": tb.value, "classes": cl.value, "energy_passes": ps.value}

    def grad_info(self) -> dict:
        """Passes over the state of sigma and of the reverse sweep."""
        a = ctypes.c_int64()
        b = ctypes.c_int64()
        check(lib.qf_plan_grad_info(self._h, ctypes.byref(a), ctypes.byref(b)), "qf_plan_grad_info")
        return {"sigma_passes": a.value, "sweep_passes": b.value}

    def set_block_bits(self, block_bits: int) -> None:
        """0: one pass per fused run; 6-12: runs applied in LDS sub-cubes of 2^B amplitudes."""
        check(lib.qf_plan_set_block_bits(self._h, int(block_bits)), "qf_plan_set_block_bits")

    def apply_info(self) -> dict:
        bb = ctypes.c_int()
        r = ctypes.c_int64()
        ps = ctypes.c_int64()
        check(lib.qf_plan_apply_info(self._h, ctypes.byref(bb), ctypes.byref(r), ctypes.byref(ps)),
              "qf_plan_apply_info")
        return {"block_bits": bb.value, "runs": r.value, "passes": ps.value}

    def apply(self, psi, theta, inverse: bool = False, stream=None) -> None:
        theta = _f64(theta)
        check(lib.qf_plan_apply(self._h, ptr(psi), ptr(theta), int(inverse), stream_handle(stream)),
              "qf_plan_apply")

    def energy(self, psi, stream=None) -> float:
        e = ctypes.c_double()
        check(lib.qf_plan_energy(self._h, ptr(psi), ctypes.byref(e), stream_handle(stream)), "qf_plan_energy")
        return e.value

    def sigma(self, psi, lam, stream=None) -> float:
        e = ctypes.c_double()
        check(lib.qf_plan_sigma(self._h, ptr(psi), ptr(lam), ctypes.byref(e), stream_handle(stream)),
              "qf_plan_sigma")
        return e.value

    def trotter(self, psi, t: float, r: int, stream=None) -> None:
        """qf_plan_trotter: psi <- (prod_l exp(-i t h_l P_l / r))^r psi over
        the plan's ansatz strings (a plan made with the Hamiltonian as ansatz)."""
        check(lib.qf_plan_trotter(self._h, ptr(psi), float(t), int(r), stream_handle(stream)), "qf_plan_trotter")

    def qk_matrices(self, occ_mask: int, dt: float, s: int, r: int, states=None, stream=None):
        """qf_plan_qk_matrices: (S, Hm) complex (s+1) x (s+1) for the basis
        psi_k = Trotter(k dt, r)|occ> (Sec. 3.7).  states: complex128 tensor
        of (s + 2) * 2^n (allocated if None); returns states too."""
        import torch
        if states is None:
            states = torch.empty((s + 2) << self.n, dtype=torch.complex128, device="cuda")
        S = np.zeros((s + 1, s + 1), dtype=np.complex128)
        Hm = np.zeros_like(S)
        check(lib.qf_plan_qk_matrices(self._h, occ_mask, float(dt), int(s), int(r), ptr(states), ptr(S), ptr(Hm),
                                      stream_handle(stream)), "qf_plan_qk_matrices")
        return S, Hm, states

    def pqe_residuals(self, occ_mask: int, theta, det, sign, workspace, stream=None):
        """qf_plan_pqe_residuals: (E, r), r_mu = <Phi_mu|U^dagger H U|Phi_0>."""
        theta = _f64(theta)
        det = np.ascontiguousarray(det, dtype=np.uint64)
        sign = np.ascontiguousarray(sign, dtype=np.int32)
        e = ctypes.c_double()
        r = np.zeros(len(det), dtype=np.float64)
        check(lib.qf_plan_pqe_residuals(self._h, occ_mask, ptr(theta), ptr(det), ptr(sign), len(det), ptr(workspace),
                                        ctypes.byref(e), ptr(r), stream_handle(stream)), "qf_plan_pqe_residuals")
        return e.value, r

    def pqe_solve(self, occ_mask: int, exc_off, det, sign, delta, t0, workspace, max_iter: int = 100,
                  tol: float = 1e-8, stream=None):
        """qf_plan_pqe_solve: fixed-point PQE (Eq. (fixed_point)) from t0.
        Returns (t, E, r, updates)."""
        exc_off = np.ascontiguousarray(exc_off, dtype=np.int64)
        t = np.array(t0, dtype=np.float64)
        det = np.ascontiguousarray(det, dtype=np.uint64)
        sign = np.ascontiguousarray(sign, dtype=np.int32)
        delta = _f64(delta)
        e = ctypes.c_double()
        r = np.zeros(len(t), dtype=np.float64)
        it = ctypes.c_int()
        check(lib.qf_plan_pqe_solve(self._h, occ_mask, ptr(self._A), ptr(exc_off), len(t), ptr(det), ptr(sign),
                                    ptr(delta), ptr(t), int(max_iter), float(tol), ptr(workspace), ctypes.byref(e),
                                    ptr(r), ctypes.byref(it), stream_handle(stream)), "qf_plan_pqe_solve")
        return t, e.value, r, it.value

    def pool_grad(self, pool: "PoolPlan", occ_mask: int, theta, workspace, stream=None):
        """qf_plan_pool_grad: (E, g) for the pool members (ADAPT-VQE, Sec. 3.2)."""
        theta = _f64(theta)
        e = ctypes.c_double()
        g = np.zeros(pool.n_pool, dtype=np.float64)
        check(lib.qf_plan_pool_grad(self._h, pool._h, occ_mask, ptr(theta), ptr(workspace), ctypes.byref(e),
                                    ptr(g), stream_handle(stream)), "qf_plan_pool_grad")
        return e.value, g

    def energy_grad(self, occ_mask: int, theta, workspace, stream=None):
        theta = _f64(theta)
        e = ctypes.c_double()
        g = np.zeros(self.K, dtype=np.float64)
        check(lib.qf_plan_energy_grad(self._h, occ_mask, ptr(theta), ptr(workspace), ctypes.byref(e), ptr(g),
                                      stream_handle(stream)), "qf_plan_energy_grad")
        return e.value, g


class Batch:
    """qf_batch_*: many instances' energy + adjoint gradient in one persistent launch.

    instances: list of dicts with keys n (qubits), occ (int mask), A (ansatz
    terms), H (Hamiltonian terms), off (group offsets).  team: optional list
    of workgroups per instance (<= 0: library default); None uses the
    autotuned table for this device when one is committed.
    """

    def __init__(self, instances, team=None):
        self.count = len(instances)
        self._keep = []
        n = (ctypes.c_int * self.count)(*[int(d["n"]) for d in instances])
        occ = (ctypes.c_uint64 * self.count)(*[int(d["occ"]) for d in instances])
        self.K = [0 if d["A"] is None else len(d["A"]) for d in instances]
        K = (ctypes.c_int64 * self.count)(*self.K)
        offs = [np.ascontiguousarray(d["off"], dtype=np.int64) for d in instances]
        self._keep += [d["A"] for d in instances] + [d["H"] for d in instances] + offs
        A = (ctypes.c_void_p * self.count)(*[ptr(d["A"]) for d in instances])
        H = (ctypes.c_void_p * self.count)(*[ptr(d["H"]) for d in instances])
        O = (ctypes.c_void_p * self.count)(*[ptr(o) for o in offs])
        G = (ctypes.c_int64 * self.count)(*[len(o) - 1 for o in offs])
        if team is None:
            from .autotune import device_arch, load_table
            tab = load_table(device_arch())
            if tab:
                team = [tab.get(int(d["n"]), 0) for d in instances]
        T = None if team is None else (ctypes.c_int * self.count)(*[int(w) for w in team])
        h = ctypes.c_void_p()
        check(lib.qf_batch_create(self.count, n, occ, A, K, H, O, G, T, ctypes.byref(h)), "qf_batch_create")
        self._h = h
        self.koff = np.concatenate([[0], np.cumsum(self.K)]).astype(np.int64)

    def close(self, _destroy=lib.qf_batch_destroy):
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def info(self):
        team = (ctypes.c_int * self.count)()
        sb = ctypes.c_int64()
        grid = ctypes.c_int()
        check(lib.qf_batch_info(self._h, team, ctypes.byref(sb), ctypes.byref(grid)), "qf_batch_info")
        return {"team": list(team), "state_bytes": sb.value, "grid": grid.value}

    def status(self) -> list:
        """Per-instance status of the last completed launch: 0 (QF_OK) or -4
        (QF_E_HIP: that instance's team barrier timed out)."""
        st = (ctypes.c_int * self.count)()
        check(lib.qf_batch_status(self._h, st), "qf_batch_status")
        return list(st)

    def set_spin_limit(self, polls: int):
        check(lib.qf_batch_set_spin_limit(self._h, int(polls)), "qf_batch_set_spin_limit")

    def run(self, thetas, use_graph: bool = True, stream=None, partial: bool = False):
        """thetas: list of per-instance angle arrays.  Returns (E[count], [grad_i]).
        partial: do not raise when only some instances failed (team barrier
        timeouts); return (E, grads, status) with status as in status()."""
        theta = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.float64) for t in thetas])
                                     if self.count else np.zeros(0), dtype=np.float64)
        if len(theta) != self.koff[-1]:
            raise ValueError("theta lengths do not match the batch's ansatz sizes")
        E = np.zeros(self.count)
        g = np.zeros(max(len(theta), 1))
        st = lib.qf_batch_run(self._h, ptr(theta), ptr(E), ptr(g), int(use_graph), stream_handle(stream))
        grads = [g[self.koff[i]:self.koff[i + 1]].copy() for i in range(self.count)]
        if partial:
            status = self.status()
            if st != _lib.QF_OK and all(v == _lib.QF_OK for v in status):
                check(st, "qf_batch_run")
            return E, grads, status
        check(st, "qf_batch_run")
        return E, grads

    def run_completion(self, thetas, stream=None, poll_s: float = 20e-6):
        """One launch in which the kernel publishes each instance to a host
        mailbox as soon as its team finishes (qf_batch_launch_mailbox).
        Returns (E, grads, t_done): t_done[i] is the time in seconds from the
        launch call to the host seeing instance i's flag."""
        import time
        theta = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.float64) for t in thetas])
                                     if self.count else np.zeros(0), dtype=np.float64)
        if len(theta) != self.koff[-1]:
            raise ValueError("theta lengths do not match the batch's ansatz sizes")
        need = ctypes.c_int64()
        check(lib.qf_batch_mailbox_bytes(self._h, ctypes.byref(need)), "qf_batch_mailbox_bytes")
        mb = ctypes.c_void_p()
        check(lib.qf_mailbox_alloc(need.value, ctypes.byref(mb)), "qf_mailbox_alloc")
        try:
            kt = int(self.koff[-1])
            flags = np.ctypeslib.as_array(
                ctypes.cast(ctypes.c_void_p(mb.value + 8 * self.count + 8 * kt), ctypes.POINTER(ctypes.c_uint32)),
                shape=(self.count,))
            t_done = np.full(self.count, np.nan)
            t0 = time.perf_counter()
            check(lib.qf_batch_launch_mailbox(self._h, ptr(theta), mb, need.value, stream_handle(stream)),
                  "qf_batch_launch_mailbox")
            while True:
                now = time.perf_counter() - t0
                up = (flags == 1) & np.isnan(t_done)
                t_done[up] = now
                if not np.isnan(t_done).any() or lib.qf_batch_poll(self._h) == 0:
                    break
                time.sleep(poll_s)
            E = np.zeros(self.count)
            g = np.zeros(max(kt, 1))
            check(lib.qf_batch_collect(self._h, ptr(E), ptr(g)), "qf_batch_collect")
            t_done[np.isnan(t_done)] = time.perf_counter() - t0
        finally:
            lib.qf_mailbox_free(mb)
        return E, [g[self.koff[i]:self.koff[i + 1]].copy() for i in range(self.count)], t_done
