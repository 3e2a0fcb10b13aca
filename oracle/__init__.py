"""CPU oracle for the subspace-Hamiltonian SpMV (test infrastructure, not product code).

A plain, slow, obviously-correct implementation of what the GPU path computes, written
from the paper's definitions.  It shares no code with the GPU library
(``paper_2603_18731_amd``) and never imports it.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import, call or link anything here.

Routes (each independent of the others and of the GPU path):

* ``alphabet`` - the seven single-qubit matrices of the extended alphabet (Methods,
  Qubit Hamiltonians) in the basis ``|0>, |1>``.
* ``dense``    - Kronecker-product Hamiltonians for ``n <= 14`` and their restriction to a
  subspace; exact diagonalization by LAPACK.
* ``fermion``  - dense Jordan-Wigner fermion matrices, and the direct second-quantized
  action of a product of ladder operators on a bit-string (any ``n``).
* ``subspace`` - canonical index: ascending unsigned integer order after dedup
  (Lower / upper triangle evaluation section).
* ``rowwise``  - term-by-term row evaluation (no grouping, no ladder integers, no hashing;
  binary search for columns), in Python for tiny cases and in plain C with OpenMP
  (``csrc/qsd_oracle.c``) for sampled rows at full size.
* ``lanczos``  - CPU Lanczos with full reorthogonalization, ``numpy.linalg.eigh`` on T.
* ``closed_forms`` - textbook ground energies used as pins.

Readings of silent or ambiguous points of the paper that this oracle adopts:

* qubit ``q`` = bit ``q`` of the integer value of the bit-string;
* ``H_ij = <b_i|H|b_j>`` with rows ``i`` and index = rank in ascending order;
* ``+ = |1><0|`` and ``- = |0><1|`` (``-`` is the JW image of ``f``);
* an off-diagonal entry ``(i, j)`` is *present* iff ``b_j`` is in the subspace and some
  input term with a nonzero coefficient has a nonzero matrix element between ``b_i`` and
  ``b_j`` (its value may cancel to 0.0); the diagonal entry is always present;
* an identity word adds its coefficient to every diagonal entry.
"""
