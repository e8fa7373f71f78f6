/*
 * qforte_mi355x.h - C ABI of the MI355X (gfx950) Pauli-exponential
 * state-vector library.
 *
 * The library implements the state-vector hot path of Stair & Evangelista,
 * "QForte: an efficient state simulator and quantum algorithms library for
 * molecular electronic structure": a molecular Hamiltonian and a
 * disentangled UCC ansatz are mapped to Pauli strings by the Jordan-Wigner
 * transformation, the ansatz is applied to a 2^n complex128 state as an
 * ordered product of Pauli-string exponentials, and <psi|H|psi> and its
 * gradient are evaluated.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Qubit q is bit q of the amplitude index (Sec. 2.1.1, Eq. (3)).  A state
 *   is 2^n complex128 values, interleaved (re, im), in DEVICE memory owned by
 *   the caller; the library never frees caller memory.
 * - A term {x, z, c} denotes c * P(x, z) with
 *       P(x, z) = i^popcount(x & z) X^x Z^z,
 *   a Hermitian Pauli string (a qubit in both masks carries Y).  Term arrays
 *   are HOST memory, read during the call only.
 * - 1 <= n_qubits <= QF_MAX_QUBITS; every mask must be < 2^n_qubits.
 * - Calls are ordered on `stream` (a hipStream_t; NULL = the default
 *   stream).  Calls that return host values synchronize that stream before
 *   returning.  Calls on distinct states and streams may run concurrently.
 * - Every call returns a qf_status; on failure qf_last_error() returns a
 *   message for the calling thread.  No C++ exception crosses this ABI.
 */
#ifndef QFORTE_MI355X_H
#define QFORTE_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QF_MAX_QUBITS 30 /* full-space states: 2^30 amplitudes = 16 GiB (tested) */

typedef struct qf_term {
    uint64_t x; /* flip mask: qubits carrying X or Y */
    uint64_t z; /* phase mask: qubits carrying Z or Y */
    double c;   /* real coefficient */
} qf_term;

typedef enum qf_status {
    QF_OK = 0,
    QF_E_ARG = -1,     /* null pointer, negative count, bad kind */
    QF_E_RANGE = -2,   /* n_qubits out of range, mask bit >= n_qubits */
    QF_E_NOMEM = -3,   /* device or host allocation failed */
    QF_E_HIP = -4,     /* a HIP runtime call failed */
    QF_E_SIZE = -5,    /* output buffer too small; sizes were written */
    QF_E_NOTHERM = -6  /* a built operator has a non-real coefficient */
} qf_status;

typedef enum qf_kind {
    QF_HAMILTONIAN = 0, /* H of Eq. (1) mapped to Eq. (2), grouped by flip mask */
    QF_UCCSD = 1,       /* kappa_mu for all S_z-conserving singles + doubles */
    QF_UCCD = 2,        /* kappa_mu for all S_z-conserving doubles */
    QF_UCCD_TOP = 3,    /* the top_k doubles by |t_rank|, canonical order */
    QF_PUCCD = 4,       /* paired (seniority-zero) doubles of Sec. 5 */
    QF_GSD_POOL = 5     /* ADAPT pool of Sec. 3.2: generalized singles + doubles */
} qf_kind;

/*
 * Build Jordan-Wigner Pauli tables on the host.
 *
 * Hamiltonian (kind QF_HAMILTONIAN), Sec. 1 Eqs. (1)-(2):
 *   H = sum_PQ h_PQ a+_P a_Q + 1/4 sum_PQRS <PQ||RS> a+_P a+_Q a_S a_R + e_core
 *   over 2*n_orb spin orbitals, spin orbital 2p = alpha and 2p+1 = beta of
 *   spatial orbital p; h is n_orb x n_orb (row-major, symmetric) and g is
 *   n_orb^4 (row-major) chemists' integrals g[p,q,r,s] = (pq|rs) with
 *   <PQ|RS> = (pr|qs) when spins of P,R and of Q,S agree.  JW of Sec. 2.2,
 *   Eqs. (13)-(14).  Like strings are summed; |Im c| > 1e-12 gives
 *   QF_E_NOTHERM; |c| <= 1e-12 is dropped.  Output is sorted by (x, z);
 *   off[] is the CSR of flip-mask groups (off[0] = 0, n_off = groups + 1).
 *
 * Ansatz kinds, Sec. 3.1 Eq. (18): for each excitation mu,
 *   kappa_mu = tau_mu - tau_mu^dagger, tau = a+_a [a+_b] [a_j] a_i,
 *   i < j occupied, a < b virtual, S_z conserved, reference = the n_elec
 *   lowest spin orbitals.  Excitations are ordered by the ascending integer
 *   value of the excited determinant; the output holds, per excitation, the
 *   strings of JW(kappa_mu) = i sum_k c_k P_k sorted by (x, z), and off[] is
 *   the excitation CSR.  exp(t kappa_mu) = prod_k exp(-i theta_k P_k) with
 *   theta_k = -c_k t_mu (see qf_ansatz_angles).
 *   QF_UCCD_TOP ranks all doubles by |t_rank[m]| (descending, ties to the
 *   lower canonical index m), keeps top_k and emits them in canonical order;
 *   t_rank has one value per double in QF_UCCD order.  kept[] (may be NULL)
 *   receives, per emitted excitation, its index in the unfiltered list.
 *   QF_GSD_POOL (n_elec ignored): the generalized pool of ADAPT-VQE
 *   (Sec. 3.2), every S_z-conserving tau = a+_p a_q with p > q (singles,
 *   ordered by (q, p)) and tau = a+_p a+_q a_s a_r with p < q, r < s,
 *   (p, q) after (r, s) lexicographically, index sets allowed to overlap
 *   (doubles, ordered by ((r, s), (p, q))); strings as for the ansatz kinds.
 *
 * Sizes: with out == NULL only *n_out and *n_off are written (QF_OK).  With
 * cap < *n_out or off_cap < *n_off the sizes are written and QF_E_SIZE is
 * returned.  h and g may be NULL for ansatz kinds.
 */
int qf_build_paulis(int kind, int n_orb, int n_elec, const double *h, const double *g,
                    double e_core, const double *t_rank, int64_t top_k,
                    qf_term *out, int64_t cap, int64_t *n_out,
                    int64_t *off, int64_t off_cap, int64_t *n_off, int64_t *kept);

/*
 * theta_k = -c_k t_mu for every string k of excitation mu (Sec. 3.1,
 * Eq. (18) written as a product of exponentials exp(-i theta_k P_k)).
 * All arrays are host memory; exc_off has n_par + 1 entries.
 */
int qf_ansatz_angles(const qf_term *A, const int64_t *exc_off, int64_t n_par,
                     const double *t, double *theta);

/* dE/dt_mu = -sum_{k in mu} c_k dE/dtheta_k (chain rule of qf_ansatz_angles). */
int qf_grad_t(const qf_term *A, const int64_t *exc_off, int64_t n_par,
              const double *dE_dtheta, double *dE_dt);

/*
 * psi <- |occ_mask>: the reference determinant Phi_0 (Sec. 3.1), one write
 * pass over the 2^n_qubits device amplitudes.
 */
int qf_prepare_state(void *psi, int n_qubits, uint64_t occ_mask, void *stream);

/*
 * psi <- U psi with U = exp(-i theta_{K-1} P_{K-1}) ... exp(-i theta_0 P_0)
 * (term 0 acts first; the c field of each term is ignored).  inverse != 0
 * applies U^dagger instead.  Each exponential is cos(theta) - i sin(theta) P
 * (Sec. 2.1.4, Eq. (8) with the sign of the worked example, Eqs. (10)-(11)).
 * Consecutive terms with the same flip mask that commute are applied in one
 * pass over the state.  theta is host memory (K values).
 */
int qf_apply_pauli_exp(void *psi, int n_qubits, const qf_term *terms, const double *theta,
                       int64_t K, int inverse, void *stream);

/*
 * *E_out = <psi|H|psi> = sum_l c_l <psi|P_l|psi> (Sec. 3.1, Eq. (17);
 * Sec. 2.2 exact operator averaging).  H is grouped by flip mask: group g
 * holds H[group_off[g] .. group_off[g+1]) and every string in it has the
 * same x.  The reduction order is fixed, so results are reproducible.
 */
int qf_energy(const void *psi, int n_qubits, const qf_term *H, const int64_t *group_off,
              int64_t n_groups, double *E_out, void *stream);

/*
 * qf_energy for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, hosts that forbid hipMalloc): the
 * same result from the same kernels, with every device table and scratch
 * array carved from a 16 MiB static device array that the library holds on
 * each GPU until the process ends (Hamiltonians up to 30 qubits fit; larger
 * tables give QF_E_SIZE).  The call performs no hipMalloc, hipFree or other
 * allocating device call.  All calls on one GPU share that array and leave
 * it holding their tables: calls that overlap on one GPU (two host threads,
 * two streams) race and must be serialized by the caller.
 */
int qf_energy_static(const void *psi, int n_qubits, const qf_term *H, const int64_t *group_off,
                     int64_t n_groups, double *E_out, void *stream);

/*
 * Energy E(theta) = <Phi|U^dagger H U|Phi> (Sec. 3.1, Eq. (16)) with
 * U from qf_apply_pauli_exp and Phi = |occ_mask>, and its gradient
 * dE_dtheta[k] = dE/dtheta_k = 2 Im <lambda_k|P_k|phi_k> by one reverse
 * sweep (phi_k = U_k..U_0 Phi, lambda_k = U_{k+1}^dagger..U_{K-1}^dagger H psi).
 * workspace: device memory of at least 2 * 2^n_qubits * 16 bytes, owned by
 * the caller.  E_out and dE_dtheta (K values) are host memory.
 */
int qf_energy_grad(int n_qubits, uint64_t occ_mask, const qf_term *A, const double *theta,
                   int64_t K, const qf_term *H, const int64_t *group_off, int64_t n_groups,
                   void *workspace, double *E_out, double *dE_dtheta, void *stream);

/*
 * Plans: device-resident copies of an ansatz and/or a Hamiltonian for
 * repeated calls (the one-shot calls above build and free one per call).
 * A may be NULL with K = 0; H may be NULL with n_groups = 0.  A plan may be
 * used from one stream at a time.
 */
typedef struct qf_plan qf_plan;

int qf_plan_create(int n_qubits, const qf_term *A, int64_t K, const qf_term *H,
                   const int64_t *group_off, int64_t n_groups, qf_plan **out);
/*
 * A plan whose device tables live in the caller's device buffer `arena`
 * (256-byte aligned, arena_bytes long, owned by the caller; the plan never
 * frees it), for serving loops that must not allocate or free device memory
 * while other work runs.  *need_bytes receives the bytes the tables need;
 * with arena == NULL nothing else happens (size query, QF_OK); a smaller
 * arena gives QF_E_SIZE.  Tables are uploaded on `stream` before the call
 * returns.  block_bits and energy_tile fix the apply blocking and the energy
 * tile as qf_plan_set_block_bits and qf_plan_set_energy_tile (merged) would
 * (< 0: the defaults); the two setters reject arena plans.
 * qf_plan_destroy releases the plan's host memory only.
 */
int qf_plan_create_arena(int n_qubits, const qf_term *A, int64_t K, const qf_term *H,
                         const int64_t *group_off, int64_t n_groups, int block_bits, int energy_tile,
                         void *arena, int64_t arena_bytes, int64_t *need_bytes, void *stream, qf_plan **out);
int qf_plan_destroy(qf_plan *plan);
/* as qf_apply_pauli_exp with the plan's ansatz */
int qf_plan_apply(qf_plan *plan, void *psi, const double *theta, int inverse, void *stream);
/* as qf_energy with the plan's Hamiltonian */
int qf_plan_energy(qf_plan *plan, const void *psi, double *E_out, void *stream);
/* as qf_energy_grad with the plan's ansatz and Hamiltonian */
int qf_plan_energy_grad(qf_plan *plan, uint64_t occ_mask, const double *theta, void *workspace,
                        double *E_out, double *dE_dtheta, void *stream);
/*
 * Energy kernel of a plan.  tile_bits = 0: one pass over the state per
 * flip-mask group.  tile_bits = L in {10, 11, 12}: groups whose flip masks
 * agree above bit L form a class; one pass per class visits pairs of tiles
 * of 2^L amplitudes (t, t ^ x_high) with the partner tile staged in LDS and
 * evaluates every group of the class, so the state is read once per class.
 * merged != 0 additionally folds each string's sign from the bits above the
 * tile into a per-tile coefficient, so strings of a group that agree below
 * bit L are evaluated once.  Plans with n_qubits >= 16 default to L = 11,
 * merged.  Needs n_qubits > L.
 */
int qf_plan_set_energy_tile(qf_plan *plan, int tile_bits, int merged);
/* tile bits (negative when merged), number of classes, passes over the
 * state per energy evaluation */
int qf_plan_info(const qf_plan *plan, int *tile_bits, int64_t *classes, int64_t *energy_passes);

/*
 * Forward application of a plan's ansatz.  block_bits = 0: one pass over
 * the state per fused run.  block_bits = B in 6..min(12, n_qubits):
 * consecutive runs whose flip masks fit, together with the lowest qubits, in
 * a set of B qubits form a segment; each segment is one pass in which every
 * sub-cube of 2^B amplitudes is loaded into LDS, updated by all the
 * segment's runs in order, and stored.  Default: B = min(12, n_qubits) for
 * n_qubits >= 6.  The reverse sweep of qf_plan_energy_grad follows: for
 * B >= 10 it undoes segments on sub-cubes of min(B, 11) qubits of phi and
 * lambda (Sec. 3.1 gradient, one pass per segment), otherwise one pass per
 * fused run.  The Python binding applies autotuned values of B and of the
 * energy tile per qubit count when its table matches the device.
 */
int qf_plan_set_block_bits(qf_plan *plan, int block_bits);
/* passes over the state of the plan's sigma (lambda = H psi: one per class
 * of 2^11-amplitude tiles from 12 qubits up, else one per group, each
 * reading psi) and of its reverse sweep (one per segment, or per run below
 * 10 block bits) */
int qf_plan_grad_info(const qf_plan *plan, int64_t *sigma_passes, int64_t *sweep_passes);
/* block bits, number of fused runs, passes over the state per application */
int qf_plan_apply_info(const qf_plan *plan, int *block_bits, int64_t *runs, int64_t *passes);
/* lambda <- H psi and *E_out = Re <psi|lambda> (device states, host E_out).
 * For n_qubits >= 12 the groups are taken in classes by their flip bits
 * above bit 11 and each class's partner tile of 2^11 amplitudes is read once
 * per output tile; below, psi[y ^ x] is gathered per group. */
int qf_plan_sigma(qf_plan *plan, const void *psi, void *lambda, double *E_out, void *stream);

/*
 * ADAPT-VQE pool gradients (Sec. 3.2).  For Psi = U(theta)|occ_mask> (U as
 * in qf_apply_pauli_exp) and each pool member nu with JW(kappa_nu) =
 * i sum_k c_k P_k (strings pool[pool_off[nu] .. pool_off[nu+1]), one flip
 * mask per member, e.g. from qf_build_paulis(QF_GSD_POOL)):
 *   g_nu = <Psi|[H, kappa_nu]|Psi> = 2 Re <H Psi|kappa_nu Psi>
 *        = -sum_k c_k 2 Im <H Psi|P_k|Psi>,
 * the derivative of the energy with respect to t of exp(t kappa_nu)
 * appended to the ansatz, at t = 0.  One forward pass, lambda = H Psi, then
 * read-only passes over (Psi, lambda) that evaluate every pool string.
 * workspace: 2 * 2^n_qubits * 16 bytes of device memory (Psi, lambda; on
 * return they hold Psi and H Psi).  E_out (the energy) and g_out (n_pool
 * values, caller order) are host memory.
 * qf_plan_create_pool makes a plan of a pool for repeated calls;
 * qf_plan_pool_grad takes a plan holding the ansatz and Hamiltonian and a
 * pool plan of the same qubit count.
 */
int qf_pool_grad(int n_qubits, uint64_t occ_mask, const qf_term *A, const double *theta, int64_t K,
                 const qf_term *H, const int64_t *group_off, int64_t n_groups, const qf_term *pool,
                 const int64_t *pool_off, int64_t n_pool, void *workspace, double *E_out, double *g_out,
                 void *stream);
int qf_plan_create_pool(int n_qubits, const qf_term *pool, const int64_t *pool_off, int64_t n_pool,
                        qf_plan **out);
int qf_plan_pool_grad(qf_plan *plan, qf_plan *pool, uint64_t occ_mask, const double *theta, void *workspace,
                      double *E_out, double *g_out, void *stream);

/*
 * PQE (Sec. 3.3).  qf_excited_determinants: for each excitation of an
 * ansatz kind, in qf_build_paulis order, the excited determinant
 * tau_mu |ref> = sign[mu] |det[mu]> (bit strings; sign 0 if tau_mu
 * annihilates the reference, which particle-hole kinds never do); with
 * det == NULL only *n_out is written.  qf_mp_denominators: the
 * Moller-Plesset denominators Delta_mu = sum eps_occ - sum eps_vir of the
 * particle-hole kinds, with eps_P the diagonal of the reference's Fock
 * matrix, h_pp + sum_{J occupied} <PJ||PJ> (the reading for references that
 * are not canonical Hartree-Fock determinants).
 * qf_pqe_residuals / qf_plan_pqe_residuals: for Psi = U(theta)|occ_mask>,
 *   r_mu = <Phi_mu|U^dagger H U|Phi_0> = sign[mu] [U^dagger H Psi](det[mu])
 * (Eq. (ucc2)) for n_res <= K determinants: one forward pass, lambda = H Psi,
 * the ansatz undone on lambda in reverse, and the amplitudes at det[] (the
 * real part; U and H are real).  E_out receives <Psi|H|Psi>.  workspace:
 * 2 * 2^n_qubits * 16 bytes of device memory.  det, sign, r_out: host.
 * qf_plan_pqe_solve: the fixed-point iteration of Eq. (fixed_point),
 *   t_mu <- t_mu + r_mu / Delta_mu,
 * from t (host, n_par amplitudes, updated in place) until max |r_mu| < tol
 * or max_iter updates; theta_k = -c_k t_mu as qf_ansatz_angles.  r_out
 * holds the last residuals, *iters the number of updates made.
 */
int qf_excited_determinants(int kind, int n_orb, int n_elec, const double *t_rank, int64_t top_k,
                            uint64_t *det, int *sign, int64_t cap, int64_t *n_out);
int qf_mp_denominators(int kind, int n_orb, int n_elec, const double *h, const double *g,
                       const double *t_rank, int64_t top_k, double *delta, int64_t cap, int64_t *n_out);
int qf_pqe_residuals(int n_qubits, uint64_t occ_mask, const qf_term *A, const double *theta, int64_t K,
                     const qf_term *H, const int64_t *group_off, int64_t n_groups, const uint64_t *det,
                     const int *sign, int64_t n_res, void *workspace, double *E_out, double *r_out, void *stream);
int qf_plan_pqe_residuals(qf_plan *plan, uint64_t occ_mask, const double *theta, const uint64_t *det,
                          const int *sign, int64_t n_res, void *workspace, double *E_out, double *r_out,
                          void *stream);
int qf_plan_pqe_solve(qf_plan *plan, uint64_t occ_mask, const qf_term *A, const int64_t *exc_off, int64_t n_par,
                      const uint64_t *det, const int *sign, const double *delta, double *t, int max_iter,
                      double tol, void *workspace, double *E_out, double *r_out, int *iters, void *stream);

/*
 * Quantum Krylov basis by Trotterized real-time evolution (Sec. 3.7).
 * The plan must hold the Hamiltonian twice: as its ansatz (A = H's strings
 * with their coefficients h_l, in the order of the product) and as its
 * grouped Hamiltonian (qf_plan_create(n, H, K_H, H, group_off, G)).
 * qf_plan_trotter: psi <- (prod_l exp(-i t h_l P_l / r))^r psi
 *   (Eq. (m_trotter_step2); the first string acts first; r >= 1).
 * qf_plan_qk_matrices: the basis psi_k = Trotter(k dt, r)|occ_mask>,
 *   k = 0 .. s (0 <= s < 16), each evolved from the reference, and
 *   S_out[m][k] = <psi_m|psi_k>, H_out[m][k] = <psi_m|H|psi_k>
 *   ((s+1)^2 complex values each, row-major, interleaved re/im, host).
 *   states: device memory for s + 2 states ((s+2) * 2^n_qubits * 16 bytes);
 *   on return states[k] holds psi_k.  The generalized eigenproblem
 *   H c = S c E is left to the caller.
 */
int qf_plan_trotter(qf_plan *plan, void *psi, double t, int r, void *stream);
int qf_plan_qk_matrices(qf_plan *plan, uint64_t occ_mask, double dt, int s, int r, void *states,
                        double *S_out, double *H_out, void *stream);

/*
 * qf_excitations: the operators of each excitation of an ansatz kind, in
 * qf_build_paulis order: ops[4 mu .. 4 mu + 3] = (c0, c1, a0, a1) for
 * tau_mu = a+_{c0} a+_{c1} a_{a0} a_{a1} (spin orbitals; -1 in the unused
 * slots of a single).  With ops == NULL only *n_out is written.
 */
int qf_excitations(int kind, int n_orb, int n_elec, const double *t_rank, int64_t top_k, int32_t *ops,
                   int64_t cap, int64_t *n_out);

/*
 * Particle-number and S_z restricted state vector (the restriction Sec. 6
 * names for going past ~24 qubits).  Only determinants with n_alpha alpha
 * and n_beta beta electrons are stored: an alpha (beta) string is the
 * n_orb-bit mask of the occupied alpha (beta) orbitals (spin orbital 2j is
 * alpha, 2j + 1 beta of spatial orbital j), strings of one spin are ranked
 * in increasing order, and determinant (a, b) is element
 * rank(a) * D_beta + rank(b) of a complex128 device vector of
 * dim = C(n_orb, n_alpha) C(n_orb, n_beta) entries (caller-owned).
 * qf_sector_create: n_orb <= 20; exc (4 ints per excitation, as from
 *   qf_excitations; may be NULL with n_exc = 0) for the dUCC factors of
 *   Sec. 3.1 Eq. (ducc), each conserving N_alpha and N_beta; H grouped by flip
 *   mask as for qf_energy (may be NULL with n_groups = 0).  Host arrays are
 *   read during the call; the sector holds its own device tables.
 * qf_sector_info: dim, D_alpha, D_beta, and the number of Hamiltonian groups
 *   that can map sector determinants onto sector determinants.
 * qf_sector_prepare: psi = |occ_mask> (a spin-orbital bit string in the
 *   sector).
 * qf_sector_apply: psi <- prod_mu exp(t_mu kappa_mu) psi (the first
 *   excitation acts first; inverse != 0 applies the adjoint in reverse):
 *   each determinant D with tau_mu D = s D' is rotated with D',
 *   D -> cos t D + s sin t D'.  t: host, one amplitude per excitation.
 * qf_sector_energy: <psi|H|psi> as the grouped Pauli sum of Eq. (17) over
 *   pairs of sector determinants (host E_out; the stream is synchronized).
 * qf_sector_energy_grad: E(t) = <Phi|U^dagger H U|Phi> for Phi = |occ_mask>
 *   and its gradient dE_dt[mu] = dE/dt_mu (Sec. 3.1, Eq. (16)), by
 *   lambda = H psi in the sector and one reverse sweep over the factors:
 *   dE/dt_mu = 2 Re <lambda_mu|kappa_mu|phi_mu>, then phi and lambda undo
 *   factor mu.  workspace: 2 * dim complex128 device values (phi, lambda);
 *   E_out and dE_dt (one value per excitation) are host memory.
 */
typedef struct qf_sector qf_sector;
int qf_sector_create(int n_orb, int n_alpha, int n_beta, const int32_t *exc, int64_t n_exc, const qf_term *H,
                     const int64_t *group_off, int64_t n_groups, qf_sector **out);
int qf_sector_info(const qf_sector *sector, int64_t *dim, int64_t *d_alpha, int64_t *d_beta, int64_t *groups);
int qf_sector_prepare(qf_sector *sector, void *psi, uint64_t occ_mask, void *stream);
int qf_sector_apply(qf_sector *sector, void *psi, const double *t, int inverse, void *stream);
int qf_sector_energy(qf_sector *sector, const void *psi, double *E_out, void *stream);
int qf_sector_energy_grad(qf_sector *sector, uint64_t occ_mask, const double *t, void *workspace, double *E_out,
                          double *dE_dt, void *stream);
int qf_sector_destroy(qf_sector *sector);

/*
 * Batches: energy and adjoint gradient of many instances (different
 * molecules, qubit counts or parameter vectors) in ONE persistent kernel
 * launch, optionally replayed as a HIP graph.  Sec. 3.1, Eqs. (16)-(18)
 * per instance, as qf_energy_grad.
 *
 * qf_batch_create: count instances; instance i has n_qubits[i] (<= 30),
 *   occ_mask[i], ansatz A[i] (K[i] strings, host), grouped Hamiltonian H[i]
 *   with group_off[i] (n_groups[i] groups, host).  team (may be NULL) gives
 *   the number of workgroups that cooperate on instance i (clamped to the
 *   resident grid and to one 2^11-amplitude sub-cube per workgroup, i.e.
 *   2^(n-11)); NULL, or team[i] == 0, uses the built-in table (2^(n-14)
 *   workgroups, 1..256); team[i] < 0 shares the resident grid among those
 *   instances in proportion to 2^n (K + Hamiltonian strings), at most
 *   2^(n-12) and at least -team[i] workgroups each (for latency when few
 *   instances are in flight).
 *   The batch owns all device memory: tables, two states per
 *   instance, outputs.  Results of an instance depend only on the instance
 *   and its team size, so they are identical alone and in any batch.
 * qf_batch_run: theta is host memory, the instances' K[i] angles
 *   concatenated in instance order; E_out[count] and dE_dtheta (same layout
 *   as theta, may be NULL) are host memory, valid on return.  use_graph != 0
 *   captures the launch (theta upload, counter reset, persistent kernel,
 *   result copies) into a HIP graph on the first call and replays it after.
 *   A team barrier that waits longer than the spin limit sets that
 *   instance's error flag: its members stop waiting, the kernel still
 *   exits, the other instances complete normally, and the call returns
 *   QF_E_HIP after writing every output; qf_batch_status tells which
 *   instances failed (their outputs are meaningless).
 * qf_batch_status: per-instance status of the last completed launch
 *   (count ints, caller order): QF_OK or QF_E_HIP.
 * qf_batch_info: per-instance team sizes (count ints), device state bytes,
 *   persistent grid size; any output may be NULL.
 * qf_batch_set_spin_limit: polls before a team barrier gives up (default 2^28).
 */
typedef struct qf_batch qf_batch;

int qf_batch_create(int count, const int *n_qubits, const uint64_t *occ_mask, const qf_term *const *A,
                    const int64_t *K, const qf_term *const *H, const int64_t *const *group_off,
                    const int64_t *n_groups, const int *team, qf_batch **out);
int qf_batch_run(qf_batch *batch, const double *theta, double *E_out, double *dE_dtheta, int use_graph,
                 void *stream);
int qf_batch_info(const qf_batch *batch, int *team, int64_t *state_bytes, int *grid);
int qf_batch_status(const qf_batch *batch, int *status);
/* Workgroups of the persistent batched kernel resident on the current device
 * (the grid of a launch with at least that many tickets). */
int qf_batch_resident_grid(int *grid);
/*
 * The team sizes qf_batch_create(_arena) would give (host only, no device):
 * n_strings[i] is instance i's Hamiltonian string count, team as above,
 * grid the resident workgroup count, concurrent as in qf_batch_create_arena.
 */
int qf_batch_teams(int count, const int *n_qubits, const int64_t *K, const int64_t *n_strings,
                   const int *team, int grid, int concurrent, int *W_out);

/*
 * Arena batches, for serving loops that must not allocate or free device
 * memory while other work runs (hipFree synchronizes the device).
 * qf_batch_create_arena: as qf_batch_create, but every device array
 *   (tables, two states per instance, outputs) is laid out in the caller's
 *   device buffer `arena` (256-byte aligned, arena_bytes long, owned by the
 *   caller and not freed by the batch).  *need_bytes receives the size the
 *   batch needs; with arena == NULL nothing else happens (size query, QF_OK);
 *   a smaller arena gives QF_E_SIZE.  Tables are uploaded on `stream` before
 *   the call returns.  concurrent (>= 1) is the number of persistent batch
 *   launches that may run on the device at once: every team is capped at
 *   (resident grid) / concurrent workgroups, which keeps overlapping launches
 *   free of deadlock (each can always gather its waiting team).
 * qf_batch_launch: queue theta upload and the persistent kernel on `stream`
 *   and return at once.  qf_batch_poll: QF_OK when the launch has finished,
 *   1 while it runs.  qf_batch_collect: wait for it and copy E_out (count)
 *   and dE_dtheta (concatenated, may be NULL) to host memory.
 * qf_batch_run on an arena batch is launch + collect (no graph).
 */
int qf_batch_create_arena(int count, const int *n_qubits, const uint64_t *occ_mask, const qf_term *const *A,
                          const int64_t *K, const qf_term *const *H, const int64_t *const *group_off,
                          const int64_t *n_groups, const int *team, int concurrent, void *arena,
                          int64_t arena_bytes, int64_t *need_bytes, void *stream, qf_batch **out);
int qf_batch_launch(qf_batch *batch, const double *theta, void *stream);
int qf_batch_poll(qf_batch *batch);
int qf_batch_collect(qf_batch *batch, double *E_out, double *dE_dtheta);

/*
 * Per-instance completion for serving.  A mailbox is coherent pinned host
 * memory (qf_mailbox_alloc zeroes it; qf_mailbox_free releases it, which may
 * synchronize the device, so servers allocate mailboxes once).
 * qf_batch_launch_mailbox is qf_batch_launch that also makes the kernel
 * publish each instance as soon as its team finishes: layout
 *   double E[count]; double dE_dtheta[K_total]; uint32 flag[count]
 * (qf_batch_mailbox_bytes gives the size); results are written first, then
 * flag[i] = 1 with a system-scope release, so a host that reads flag[i] == 1
 * may read E[i] and the instance's gradient; flag[i] = 2 marks an instance
 * whose team barrier timed out (no valid result).  The mailbox must stay
 * untouched until the launch has finished (qf_batch_poll / collect).
 */
int qf_mailbox_alloc(int64_t bytes, void **mailbox);
int qf_mailbox_free(void *mailbox);
int qf_batch_mailbox_bytes(const qf_batch *batch, int64_t *bytes);
int qf_batch_launch_mailbox(qf_batch *batch, const double *theta, void *mailbox, int64_t mailbox_bytes,
                            void *stream);
int qf_batch_set_spin_limit(qf_batch *batch, uint32_t polls);
int qf_batch_destroy(qf_batch *batch);

/* Message for the last non-OK status returned on the calling thread. */
const char *qf_last_error(void);

/* Library version string. */
const char *qf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QFORTE_MI355X_H */
