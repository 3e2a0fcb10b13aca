"""Dense (Kronecker-product) route for small systems.

Methods, Qubit Hamiltonians: ``H = sum_i c_i W_i`` with each word a tensor product of
single-qubit operators (identity on unlisted qubits).  Qubit 0 is the least significant
tensor factor, so the matrix index of a basis state equals the integer value of its
bit-string.  The subspace Hamiltonian is the principal submatrix on the canonical index
(ascending integer order).  ``scipy.sparse.kron`` assembles the products; exact
diagonalization uses ``numpy.linalg.eigvalsh`` (LAPACK).
"""
import numpy as np
import scipy.sparse as sp

from .alphabet import MATS
from . import subspace as osub

MAX_DENSE_QUBITS = 16


def word_matrix(n: int, word) -> sp.csr_matrix:
    """``kron(W_{n-1}, ..., W_0)`` of a word ``[(qubit, code), ...]`` (distinct qubits)."""
    ops = {}
    for q, code in word:
        q = int(q)
        if q in ops:
            raise ValueError("repeated qubit index in a qubit word")
        ops[q] = MATS[int(code)]
    m = sp.identity(1, dtype=np.complex128, format="csr")
    for q in range(n - 1, -1, -1):
        f = ops.get(q, np.eye(2, dtype=np.complex128))
        m = sp.kron(m, sp.csr_matrix(f), format="csr")
    return m


def qubit_hamiltonian(n: int, terms) -> sp.csr_matrix:
    """Full ``2^n x 2^n`` sparse matrix of ``[(coef, word), ...]``."""
    if n > MAX_DENSE_QUBITS:
        raise ValueError("dense route is limited to %d qubits" % MAX_DENSE_QUBITS)
    H = sp.csr_matrix((1 << n, 1 << n), dtype=np.complex128)
    for c, word in terms:
        if c == 0:
            continue
        H = H + c * word_matrix(n, word)
    return H.tocsr()


def restrict(H, values) -> np.ndarray:
    """Dense principal submatrix on the canonical index of the integer ``values``."""
    idx = np.asarray(osub.canonical(values), dtype=np.int64)
    Hd = H[idx][:, idx]
    return np.asarray(Hd.todense())


def ground_energy(Hs: np.ndarray) -> float:
    return float(np.linalg.eigvalsh(Hs)[0])
