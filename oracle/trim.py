"""Group trimming (Results, the CH4-dimer runs: groups whose matrix elements are small compared
with the smallest diagonal energy splitting of the subspace are removed before evaluation).

Test infrastructure only: nothing in the library imports this module.

Readings taken (the paper gives the criterion in one sentence):
* a group is the set of input terms with the same flip mask (the qubits whose bit the term
  changes: X, Y, raise and lower letters of a qubit word; every ladder operator of a fermionic
  word flips its mode, so the mask is the XOR of their modes).  Terms that flip nothing are
  diagonal and never trimmed;
* the size of a group's matrix elements is bounded by B_g = sum of |c_t| over its input terms
  (every word's matrix elements have modulus at most 1);
* the smallest diagonal energy splitting is the gap between the lowest diagonal element of the
  subspace and the next larger distinct one;
* a group is removed when B_g < tol * splitting.
"""
import numpy as np

import workloads as wl

FLIPPING = {3, 4, 5, 6}  # X, Y, lower, raise


def term_flip_mask(codes, qubits, fermionic: bool) -> int:
    m = 0
    for c, q in zip(codes, qubits):
        if fermionic:
            m ^= 1 << int(q)
        elif int(c) in FLIPPING:
            m |= 1 << int(q)
    return m


def group_bounds(tl: wl.TermList) -> dict:
    """{flip mask: sum of |c| over the input terms with that mask} for nonzero masks."""
    B = {}
    for t in range(len(tl.coef)):
        a, b = int(tl.term_ptr[t]), int(tl.term_ptr[t + 1])
        m = term_flip_mask(tl.op_code[a:b], tl.op_idx[a:b], tl.fermionic)
        if m and tl.coef[t] != 0:
            B[m] = B.get(m, 0.0) + abs(complex(tl.coef[t]))
    return B


def smallest_splitting(diag) -> float:
    d = np.unique(np.asarray(diag, dtype=np.float64))
    return float(d[1] - d[0]) if d.size > 1 else 0.0


def trim_terms(tl: wl.TermList, abs_tol: float) -> wl.TermList:
    """The term list without the terms of groups whose bound is below abs_tol."""
    B = group_bounds(tl)
    keep = []
    for t in range(len(tl.coef)):
        a, b = int(tl.term_ptr[t]), int(tl.term_ptr[t + 1])
        m = term_flip_mask(tl.op_code[a:b], tl.op_idx[a:b], tl.fermionic)
        if m == 0 or B.get(m, 0.0) >= abs_tol:
            keep.append(t)
    ptr = [0]
    idx, code = [], []
    for t in keep:
        a, b = int(tl.term_ptr[t]), int(tl.term_ptr[t + 1])
        idx.extend(tl.op_idx[a:b].tolist())
        code.extend(tl.op_code[a:b].tolist())
        ptr.append(len(idx))
    return wl.TermList(tl.n_qubits, np.asarray(ptr, dtype=np.int64), np.asarray(idx, dtype=np.int32),
                       np.asarray(code, dtype=np.uint8), np.asarray(tl.coef[keep], dtype=np.complex128), tl.fermionic)
