"""CPU oracle for the Pauli-exponential state-vector path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg use it.

It is a plain, slow FP64 implementation of what the paper's state-vector
simulator computes (Stair & Evangelista, "QForte: an efficient state simulator
and quantum algorithms library for molecular electronic structure"):

* ``pauli``       Pauli-string products with exact i^k phases and the
                  Jordan-Wigner ladder operators (Sec. 2.2, Eqs. (13)-(14)).
* ``hamiltonian`` integrals -> spin-orbital integrals -> qubit Hamiltonian
                  (Eqs. (1)-(2)), grouped by flip mask.
* ``ansatz``      particle-hole excitations, their canonical order and the
                  JW image of kappa_mu = tau_mu - tau_mu^dagger (Sec. 3.1,
                  Eq. (18)).
* ``statevec``    numpy state vector: prepare, exp(-i theta P), <P>, H|psi>,
                  the adjoint gradient and the parameter-shift gradient
                  (Eqs. (15)-(17)).
* ``dense``       dense-matrix toolkit for tiny systems: Kronecker-product
                  Pauli matrices, second quantization on determinant bit
                  strings (no Pauli algebra), exact diagonalization and the
                  gate circuit of Fig. "exp_pt" (Eqs. (10)-(11)).
* ``core``        ctypes binding of ``sv_core.c``: the same plain per-term
                  state-vector loops in C with OpenMP, for 20-28 qubits.

Conventions (readings of the paper are listed with each function):
qubit q is bit q of the amplitude index (Sec. 2.1.1, Eq. (3)); a Pauli term
(x, z, c) is c * P(x, z) with P(x, z) = i^popcount(x & z) X^x Z^z, which is
Hermitian; spin orbital 2p is alpha and 2p+1 is beta of spatial orbital p.
"""
