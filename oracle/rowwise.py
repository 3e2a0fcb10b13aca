"""Term-by-term row evaluation of ``H_S`` (the plain definition of the matrix).

Methods, Qubit Hamiltonians (properties 1-3) and Matrix evaluation: for a row bit-string
``b_i`` each term maps to one candidate column ``b_i xor offmask``; the element is the product
of the per-qubit 2x2 entries; the column counts only if it is in the subspace.  No grouping,
ladder integers or hashing: this is what those optimizations must reproduce exactly.

``rows_python`` is a pure-Python loop for tiny cases.  ``rows_c`` / ``matvec_c`` call the
plain C implementation in ``csrc/qsd_oracle.c`` (OpenMP over rows) for sampled rows at full
size.  Both return, per row, the sorted list of present columns with their values.
"""
import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp

from .alphabet import MATS
from . import fermion as ofe
from . import subspace as osub

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libqsd_oracle.so")
_SRC = os.path.join(_HERE, "csrc", "qsd_oracle.c")
_lib = None


def build_c(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_c(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int
        lib.qo_rows.argtypes = [i32, i64, P, i32, i64, P, P, P, P, P, i64, P, P, P, P, P, i32]
        lib.qo_rows.restype = i32
        lib.qo_matvec.argtypes = [i32, i64, P, i32, i64, P, P, P, P, P, i64, P, i32, P, P, i32]
        lib.qo_matvec.restype = i32
        lib.qo_max_threads.restype = i32
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().qo_max_threads())


# ------------------------------------------------------------------------ pure Python

def _qubit_row(b: int, word):
    """``(col, value)`` of one qubit word for row ``b`` or ``None``."""
    col = b
    val = 1.0 + 0.0j
    for q, code in word:
        rb = (b >> q) & 1
        cb = rb ^ (1 if code > 2 else 0)
        a = MATS[code][rb, cb]
        if a == 0:
            return None
        val *= a
        if code > 2:
            col ^= 1 << q
    return col, val


def rows_python(values, terms, fermionic: bool, rows=None):
    """Per row: sorted ``[(j, value), ...]`` with the diagonal always present.

    ``values`` are the canonical (sorted, distinct) Python ints of the subspace."""
    vals = list(values)
    pos = {v: i for i, v in enumerate(vals)}
    rows = range(len(vals)) if rows is None else rows
    out = []
    for i in rows:
        b = vals[i]
        acc = {i: 0.0 + 0.0j}
        for c, word in terms:
            if c == 0:
                continue
            if fermionic:
                r = ofe.row_action(b, word)
                if r is None:
                    continue
                col, f = r[1], r[0]
            else:
                r = _qubit_row(b, word)
                if r is None:
                    continue
                col, f = r
            j = pos.get(col)
            if j is None:
                continue
            acc[j] = acc.get(j, 0.0) + c * f
        out.append(sorted(acc.items()))
    return out


def csr_python(values, terms, fermionic: bool) -> sp.csr_matrix:
    rows = rows_python(values, terms, fermionic)
    indptr = [0]
    idx, data = [], []
    for r in rows:
        for j, v in r:
            idx.append(j)
            data.append(v)
        indptr.append(len(idx))
    N = len(list(values))
    return sp.csr_matrix((np.asarray(data, dtype=np.complex128), np.asarray(idx, dtype=np.int64),
                          np.asarray(indptr, dtype=np.int64)), shape=(N, N))


# ------------------------------------------------------------------------------ C

def _flat(tl):
    coef = np.ascontiguousarray(np.stack([tl.coef.real, tl.coef.imag], axis=1).astype(np.float64))
    return (np.ascontiguousarray(tl.term_ptr, dtype=np.int64), np.ascontiguousarray(tl.op_idx, dtype=np.int32),
            np.ascontiguousarray(tl.op_code, dtype=np.uint8), coef)


_MATS_FLAT = np.ascontiguousarray(np.stack([MATS.real, MATS.imag], axis=-1).astype(np.float64))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def rows_c(sorted_keys: np.ndarray, tl, rows=None, nthreads: int = 0):
    """Entries of the requested rows: ``(indptr, cols, vals)`` with complex ``vals``.

    ``sorted_keys`` must be canonical (see ``subspace.canonical_keys``)."""
    lib = _load()
    keys = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    N, W = keys.shape
    rows = np.arange(N, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    tp, oi, oc, cf = _flat(tl)
    nnz = np.zeros(rows.shape[0], dtype=np.int64)
    rc = lib.qo_rows(W, N, _p(keys), int(tl.fermionic), tl.n_terms, _p(tp), _p(oi), _p(oc), _p(cf), _p(_MATS_FLAT),
                     rows.shape[0], _p(rows), _p(nnz), None, None, None, nthreads)
    if rc != 0:
        raise RuntimeError("oracle qo_rows failed: %d" % rc)
    indptr = np.zeros(rows.shape[0] + 1, dtype=np.int64)
    np.cumsum(nnz, out=indptr[1:])
    cols = np.zeros(int(indptr[-1]), dtype=np.int64)
    vals = np.zeros((int(indptr[-1]), 2), dtype=np.float64)
    off = np.ascontiguousarray(indptr[:-1])
    rc = lib.qo_rows(W, N, _p(keys), int(tl.fermionic), tl.n_terms, _p(tp), _p(oi), _p(oc), _p(cf), _p(_MATS_FLAT),
                     rows.shape[0], _p(rows), _p(nnz), _p(off), _p(cols), _p(vals), nthreads)
    if rc != 0:
        raise RuntimeError("oracle qo_rows failed: %d" % rc)
    return indptr, cols, vals[:, 0] + 1j * vals[:, 1]


def csr_c(sorted_keys: np.ndarray, tl, nthreads: int = 0) -> sp.csr_matrix:
    indptr, cols, vals = rows_c(sorted_keys, tl, None, nthreads)
    N = sorted_keys.shape[0]
    return sp.csr_matrix((vals, cols, indptr), shape=(N, N))


def matvec_c(sorted_keys: np.ndarray, tl, x: np.ndarray, rows=None, nthreads: int = 0) -> np.ndarray:
    """``y[r] = sum_j H[rows[r], j] x[j]``; ``x`` is ``[N]`` or ``[N][nvec]``, complex result."""
    lib = _load()
    keys = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    N, W = keys.shape
    rows = np.arange(N, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    x = np.asarray(x)
    vec = x.ndim == 1
    X = x.reshape(N, -1)
    nvec = X.shape[1]
    xc = np.ascontiguousarray(np.stack([X.real, X.imag], axis=-1).astype(np.float64))
    y = np.zeros((rows.shape[0], nvec, 2), dtype=np.float64)
    tp, oi, oc, cf = _flat(tl)
    rc = lib.qo_matvec(W, N, _p(keys), int(tl.fermionic), tl.n_terms, _p(tp), _p(oi), _p(oc), _p(cf), _p(_MATS_FLAT),
                       rows.shape[0], _p(rows), nvec, _p(xc), _p(y), nthreads)
    if rc != 0:
        raise RuntimeError("oracle qo_matvec failed: %d" % rc)
    Y = y[..., 0] + 1j * y[..., 1]
    return Y[:, 0] if vec else Y


def canonical_keys(keys):
    return osub.canonical_keys(keys)
