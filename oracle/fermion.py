"""Fermionic operators: dense Jordan-Wigner matrices and direct second-quantized action.

Methods, Fermionic Hamiltonians: ladder operators obey ``{f_i, f_j} = 0`` and
``{f_i, f_j^dagger} = delta_ij``; the Jordan-Wigner image of the annihilator is
``f_j = 1/2 (X_j + i Y_j) Z_{j-1} ... Z_0`` (the printed "P_j" is read as ``Y_j``), i.e.
``|0><1|`` on qubit ``j`` with a ``Z`` string on every lower qubit.  A qubit in state
``|1>`` is an occupied mode.

Two routes, independent of each other:

* ``dense_mode_ops`` / ``dense_term``: sparse matrices of ``f_j`` built from Kronecker
  products, multiplied in product order (leftmost factor leftmost).
* ``apply_ops``: the action on a computational basis state,
  ``f_j |b> = (-1)^{popcount(b & (2^j - 1))} |b xor 2^j>`` if bit ``j`` of ``b`` is set
  (else 0) and ``f_j^dagger`` likewise with bit ``j`` clear.

Codes follow the term-list convention: 5 = ``f``, 6 = ``f^dagger``.
"""
import numpy as np
import scipy.sparse as sp

from .alphabet import MATS

F_ANN, F_CRE = 5, 6


def dense_mode_ops(n: int):
    """``[f_0, ..., f_{n-1}]`` as sparse ``2^n x 2^n`` matrices (qubit 0 least significant)."""
    Zm = sp.csr_matrix(MATS[0])
    Im = sp.identity(2, dtype=np.complex128, format="csr")
    low = sp.csr_matrix(MATS[5])
    out = []
    for j in range(n):
        m = sp.identity(1, dtype=np.complex128, format="csr")
        for q in range(n - 1, -1, -1):
            f = low if q == j else (Zm if q < j else Im)
            m = sp.kron(m, f, format="csr")
        out.append(m.tocsr())
    return out


def dense_term(n: int, ops, fs=None) -> sp.csr_matrix:
    """Matrix of the ordered product ``op_1 op_2 ... op_m`` (``ops = [(mode, code), ...]``)."""
    if fs is None:
        fs = dense_mode_ops(n)
    m = sp.identity(1 << n, dtype=np.complex128, format="csr")
    for q, code in ops:
        f = fs[int(q)]
        m = m @ (f if int(code) == F_ANN else f.conj().T.tocsr())
    return m.tocsr()


def dense_hamiltonian(n: int, terms) -> sp.csr_matrix:
    fs = dense_mode_ops(n)
    H = sp.csr_matrix((1 << n, 1 << n), dtype=np.complex128)
    for c, ops in terms:
        if c == 0:
            continue
        H = H + c * dense_term(n, ops, fs)
    return H.tocsr()


def apply_one(b: int, q: int, code: int):
    """``op|b> = sign |b'>`` -> ``(sign, b')`` or ``None`` when the result vanishes."""
    bit = (b >> q) & 1
    if int(code) == F_ANN:
        if not bit:
            return None
    else:
        if bit:
            return None
    below = b & ((1 << q) - 1)
    sign = -1 if (bin(below).count("1") & 1) else 1
    return sign, b ^ (1 << q)


def apply_ops(b: int, ops_right_to_left):
    """Apply a sequence of ``(mode, code)`` to ``|b>``, first element first."""
    s = 1
    for q, code in ops_right_to_left:
        r = apply_one(b, q, code)
        if r is None:
            return None
        s *= r[0]
        b = r[1]
    return s, b


def adjoint_code(code: int) -> int:
    return F_CRE if int(code) == F_ANN else F_ANN


def row_action(b_row: int, ops):
    """Row form of a term: ``<b_row| op_1 ... op_m = (op_m^+ ... op_1^+ |b_row>)^+``.

    Returns ``(sign, b_col)`` with ``<b_row|T|b_col> = sign`` or ``None``."""
    seq = [(q, adjoint_code(c)) for q, c in ops]  # op_1^+ is applied first
    return apply_ops(b_row, seq)
