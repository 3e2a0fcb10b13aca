"""MI355X-native subspace-Hamiltonian SpMV (arXiv 2603.18731, "Fulqrum" method).

Python binding of the C-ABI in ``include/qsd.h`` (``libqsd.so``, built for gfx950 by
``paper_2603_18731_amd.build``).  This module only marshals arguments: every step of the
path runs in the library's HIP kernels.  PyTorch supplies device memory and streams.

Classes mirror the paper's API names (Methods; workflow figure):

* ``Subspace``            - bit-strings -> canonical index + device hash table
* ``QubitOperator``       - terms over {Z, 0, 1, X, Y, -, +}
* ``FermionicOperator``   - products of f / f^dagger, compiled by the extended JW transform
* ``SubspaceHamiltonian`` - cached diagonal, ``matvec``, ``to_csr``, ``lanczos``
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsd.so")

QSD_OK = 0
F64, F32, C128, C64 = 0, 1, 2, 3
INDEX_I32, INDEX_I64 = 0, 1
OP_FERMIONIC, OP_CHECK_HERMITIAN, OP_FORCE_COMPLEX, OP_NO_LADDER_INT, OP_ORDER_BY_MASK = 1, 2, 4, 8, 16
OP_ORDER_BY_PARTS = 32
SUB_ASSUME_SORTED_UNIQUE = 1
V0_UNIFORM, V0_MIN_DIAG, V0_RANDOM, V0_USER = 0, 1, 2, 3
SCHED_XCD_REMAP, SCHED_SLOT_ORDER, SCHED_LOCKSTEP, SCHED_FILTER_FIRST = 1, 2, 4, 8
SCHED_ALL = 15
SCHED_HASH_LOOKUP = 16  # look columns up in the hash table even with a product map
TUNE_SCHEDULE, TUNE_LOAD, TUNE_SPLIT = 1, 2, 4
CSR_LOWER_MIRROR = 1
NOALLOC_MAX_REQUESTS, NOALLOC_MAX_TILES = 256, 65536  # limits of qsd_matvec_batched_noalloc
ERR_NAMES = {-1: "INVALID_ARG", -2: "OUT_OF_MEMORY", -3: "HIP", -4: "CAPACITY", -5: "NOT_HERMITIAN",
             -6: "NOT_CONVERGED", -7: "DTYPE", -8: "UNSUPPORTED"}

EXPORTED = [
    "qsd_last_error", "qsd_version", "qsd_max_qubits", "qsd_subspace_build", "qsd_subspace_info",
    "qsd_subspace_keys", "qsd_subspace_lookup", "qsd_subspace_probe_stats", "qsd_subspace_destroy",
    "qsd_op_compile", "qsd_op_info", "qsd_op_export", "qsd_op_destroy", "qsd_ham_create", "qsd_ham_diagonal",
    "qsd_ham_destroy", "qsd_ham_info", "qsd_ham_work_counts", "qsd_matvec", "qsd_csr_build", "qsd_lanczos_default_opts", "qsd_lanczos",
    "qsd_batch_create", "qsd_batch_footprint", "qsd_batch_add", "qsd_batch_step",
    "qsd_batch_poll", "qsd_batch_remove", "qsd_batch_destroy", "qsd_matvec_batched", "qsd_matvec_batched_noalloc",
    "qsd_block_lanczos",
    "qsd_ham_set_schedule", "qsd_ham_get_schedule", "qsd_ham_autotune", "qsd_subspace_rehash",
    "qsd_csr_create", "qsd_csr_info", "qsd_csr_export", "qsd_csr_matvec", "qsd_csr_lanczos", "qsd_csr_block_lanczos",
    "qsd_csr_destroy", "qsd_subspace_select", "qsd_ramps",
    "qsd_ham_diag_splitting", "qsd_batch_add_csr", "qsd_batch_footprint_rows", "qsd_subspace_hash_info",
]


class QsdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERR_NAMES.get(code, "ERROR"), code, msg))
        self.code = code


class TuneResult(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_uint32), ("capacity", ctypes.c_int64), ("max_load", ctypes.c_double),
                ("split", ctypes.c_int32), ("ms", ctypes.c_double), ("ms_before", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RampsInfo(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("truncated", ctypes.c_int32), ("paths", ctypes.c_int64),
                ("max_frontier", ctypes.c_int64), ("selected", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LanczosOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("v0_mode", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("spmv_dtype", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("want_vector", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("alloc", ctypes.c_void_p)]


# ----------------------------------------------------------------------- device memory

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    """``qsd_allocator``: device memory for the library's handles and scratch."""

    _fields_ = [("ctx", ctypes.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


def _torch_alloc(ctx, nbytes, stream):
    import torch

    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:  # out of memory: the library sees NULL and fails with OUT_OF_MEMORY
        return None


def _torch_free(ctx, ptr, stream):
    try:
        import torch

        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:  # interpreter shutdown: torch already torn down; the process frees it all
        pass


# PyTorch's caching allocator (the default): every byte the library holds is visible to
# torch.cuda.memory_allocated() and reusable by PyTorch after release.
TORCH_ALLOCATOR = Allocator(None, ALLOC_FN(_torch_alloc), FREE_FN(_torch_free))
_default_allocator = TORCH_ALLOCATOR


def set_default_allocator(a):
    """Allocator for handles created from now on: ``TORCH_ALLOCATOR`` (default), ``None``
    (hipMalloc / hipFree inside the library) or any ``Allocator`` (kept alive by the caller)."""
    global _default_allocator
    _default_allocator = a


def _resolve_allocator(a="default"):
    return _default_allocator if a == "default" else a


def _alloc_arg(a):
    return ctypes.c_void_p(0) if a is None else ctypes.cast(ctypes.pointer(a), ctypes.c_void_p)


class LanczosInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("ritz_residual", ctypes.c_double),
                ("explicit_residual", ctypes.c_double), ("matvec_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """The loaded ``libqsd.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libqsd.so is missing: build it with `python -m paper_2603_18731_amd.build` "
                           "(no CPU fallback exists)")
    # PyTorch's HIP runtime is loaded first so that the library binds to the same runtime (its
    # streams and memory are the ones passed in); loading the library first would bring in a
    # second runtime instance.
    import torch  # noqa: F401

    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "qsd_last_error": ([], ctypes.c_char_p),
        "qsd_version": ([], ctypes.c_int),
        "qsd_max_qubits": ([], I32),
        "qsd_subspace_build": ([P, I64, I32, U32, D, P, P, PP], ctypes.c_int),
        "qsd_subspace_info": ([P, P, P, P, P], ctypes.c_int),
        "qsd_subspace_keys": ([P, P, P], ctypes.c_int),
        "qsd_subspace_lookup": ([P, P, I64, P, P], ctypes.c_int),
        "qsd_subspace_probe_stats": ([P, P, P, P], ctypes.c_int),
        "qsd_subspace_destroy": ([P], ctypes.c_int),
        "qsd_op_compile": ([I32, I64, P, P, P, P, U32, D, PP], ctypes.c_int),
        "qsd_op_info": ([P, P, P, P, P, P], ctypes.c_int),
        "qsd_op_export": ([P, P, P, P, P, P, P], ctypes.c_int),
        "qsd_op_destroy": ([P], ctypes.c_int),
        "qsd_ham_create": ([P, P, U32, P, P, PP], ctypes.c_int),
        "qsd_ham_diagonal": ([P, P, P], ctypes.c_int),
        "qsd_ham_destroy": ([P], ctypes.c_int),
        "qsd_ham_info": ([P, P, P, P], ctypes.c_int),
        "qsd_ham_work_counts": ([P, P, P, P], ctypes.c_int),
        "qsd_matvec": ([P, I32, P, I64, P, I64, I32, P], ctypes.c_int),
        "qsd_csr_build": ([P, P, P, P, I32, I32, P, P], ctypes.c_int),
        "qsd_lanczos_default_opts": ([ctypes.POINTER(LanczosOpts)], None),
        "qsd_lanczos": ([P, ctypes.POINTER(LanczosOpts), P, P, ctypes.POINTER(LanczosInfo), P], ctypes.c_int),
        "qsd_batch_create": ([I32, I32, I32, P, PP], ctypes.c_int),
        "qsd_batch_footprint": ([P, I32, I32, P], ctypes.c_int),
        "qsd_batch_add": ([P, P, I32, ctypes.c_uint64, D, P, I64, P, P], ctypes.c_int),
        "qsd_matvec_batched": ([I32, P, P, P, P, I32, P], ctypes.c_int),
        "qsd_matvec_batched_noalloc": ([I32, P, P, P, P, I32, P], ctypes.c_int),
        "qsd_ham_set_schedule": ([P, U32], ctypes.c_int),
        "qsd_ham_get_schedule": ([P, P], ctypes.c_int),
        "qsd_ham_autotune": ([P, I32, I32, I32, U32, P, P], ctypes.c_int),
        "qsd_subspace_rehash": ([P, D, I32, P], ctypes.c_int),
        "qsd_subspace_hash_info": ([P, P, P, P], ctypes.c_int),
        "qsd_csr_create": ([P, I32, I32, U32, P, P, PP], ctypes.c_int),
        "qsd_csr_info": ([P, P, P, P], ctypes.c_int),
        "qsd_csr_export": ([P, P, P, P, P], ctypes.c_int),
        "qsd_csr_matvec": ([P, I32, P, I64, P, I64, I32, P], ctypes.c_int),
        "qsd_csr_lanczos": ([P, ctypes.POINTER(LanczosOpts), P, P, ctypes.POINTER(LanczosInfo), P], ctypes.c_int),
        "qsd_csr_block_lanczos": ([P, I32, ctypes.POINTER(LanczosOpts), P, P, ctypes.POINTER(LanczosInfo), P],
                                  ctypes.c_int),
        "qsd_csr_destroy": ([P], ctypes.c_int),
        "qsd_subspace_select": ([P, P, D, P, PP], ctypes.c_int),
        "qsd_ham_diag_splitting": ([P, P, P, P], ctypes.c_int),
        "qsd_ramps": ([P, P, I64, D, D, I32, I64, P, P, ctypes.POINTER(RampsInfo), P], ctypes.c_int),
        "qsd_block_lanczos": ([P, I32, ctypes.POINTER(LanczosOpts), P, P, ctypes.POINTER(LanczosInfo), P],
                              ctypes.c_int),
        "qsd_batch_step": ([P, I32, P], ctypes.c_int),
        "qsd_batch_add_csr": ([P, P, I32, ctypes.c_uint64, D, P, I64, P, P], ctypes.c_int),
        "qsd_batch_footprint_rows": ([I64, I32, I32, P], ctypes.c_int),
        "qsd_batch_poll": ([P, P, P, P, P, P], ctypes.c_int),
        "qsd_batch_remove": ([P, I32], ctypes.c_int),
        "qsd_batch_destroy": ([P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc: int):
    if rc != QSD_OK:
        raise QsdError(rc, lib().qsd_last_error().decode())


def _ptr(a) -> ctypes.c_void_p:
    if a is None:
        return ctypes.c_void_p(0)
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(a.data_ptr())


def _stream(stream=None) -> ctypes.c_void_p:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _device_tensor(a, dtype=None):
    import torch

    if isinstance(a, torch.Tensor):
        t = a
    else:
        arr = np.ascontiguousarray(a)
        if arr.dtype == np.uint64:
            arr = arr.view(np.int64)
        t = torch.from_numpy(arr)
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


# ----------------------------------------------------------------------------- classes

class Subspace:
    """Canonical bit-string subspace on the device (Methods, Subspace data structure)."""

    def __init__(self, bits, n_qubits: int, max_load: float = 0.0, assume_sorted_unique: bool = False, stream=None,
                 allocator="default"):
        import torch

        b = _device_tensor(bits)
        if b.dtype not in (torch.int64, torch.uint64):
            raise TypeError("bits must be 64-bit words")
        W = (n_qubits + 63) // 64
        b = b.reshape(-1, W) if b.numel() else b.reshape(0, W)
        self.n_qubits = int(n_qubits)
        h = ctypes.c_void_p()
        self._allocator = _resolve_allocator(allocator)  # its callbacks outlive the handle
        _check(lib().qsd_subspace_build(_ptr(b), b.shape[0], self.n_qubits,
                                        SUB_ASSUME_SORTED_UNIQUE if assume_sorted_unique else 0, max_load,
                                        _alloc_arg(self._allocator), _stream(stream), ctypes.byref(h)))
        self._h = h
        N, nq, Wo, C = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().qsd_subspace_info(h, ctypes.byref(N), ctypes.byref(nq), ctypes.byref(Wo), ctypes.byref(C)))
        self.N, self.W, self.capacity = N.value, Wo.value, C.value

    @property
    def handle(self):
        return self._h

    def __len__(self):
        return self.N

    def keys(self, stream=None):
        """Canonical strings, ``[N][W]`` int64 device tensor (uint64 bit patterns)."""
        import torch

        out = torch.empty((self.N, self.W), dtype=torch.int64, device="cuda")
        _check(lib().qsd_subspace_keys(self._h, _ptr(out), _stream(stream)))
        return out

    def lookup(self, q, stream=None):
        import torch

        qt = _device_tensor(q).reshape(-1, self.W)
        out = torch.empty(qt.shape[0], dtype=torch.int64, device="cuda")
        _check(lib().qsd_subspace_lookup(self._h, _ptr(qt), qt.shape[0], _ptr(out), _stream(stream)))
        return out

    @classmethod
    def _wrap(cls, handle, n_qubits: int, allocator=None):
        self = cls.__new__(cls)
        self._h = handle
        self._allocator = allocator
        self.n_qubits = int(n_qubits)
        N, nq, Wo, C = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().qsd_subspace_info(handle, ctypes.byref(N), ctypes.byref(nq), ctypes.byref(Wo), ctypes.byref(C)))
        self.N, self.W, self.capacity = N.value, Wo.value, C.value
        return self

    def select(self, mask, max_load: float = 0.0, stream=None) -> "Subspace":
        """The strings whose byte in ``mask`` (device uint8 [N]) is nonzero, as a new subspace."""
        h = ctypes.c_void_p()
        _check(lib().qsd_subspace_select(self._h, _ptr(mask), max_load, _stream(stream), ctypes.byref(h)))
        return Subspace._wrap(h, self.n_qubits, self._allocator)  # the library gives it this allocator

    def _refresh(self):
        N, nq, Wo, C = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().qsd_subspace_info(self._h, ctypes.byref(N), ctypes.byref(nq), ctypes.byref(Wo), ctypes.byref(C)))
        self.capacity = C.value

    def rehash(self, max_load: float, split: int = 0, stream=None):
        """Rebuilds the hash table for another load and the part filters for ``split`` (0: none,
        else the first qubit of the high part); lookups and SpMV results are unchanged."""
        _check(lib().qsd_subspace_rehash(self._h, max_load, int(split), _stream(stream)))
        self._refresh()

    def hash_info(self):
        """``(split qubit of the part filters, exact slot layout, product map)``."""
        sp_, ex, pm = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().qsd_subspace_hash_info(self._h, ctypes.byref(sp_), ctypes.byref(ex), ctypes.byref(pm)))
        return sp_.value, bool(ex.value), bool(pm.value)

    def probe_stats(self, stream=None):
        m, x = ctypes.c_double(), ctypes.c_int64()
        _check(lib().qsd_subspace_probe_stats(self._h, ctypes.byref(m), ctypes.byref(x), _stream(stream)))
        return m.value, x.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.qsd_subspace_destroy(h)
            self._h = None


class _Operator:
    fermionic = False

    def __init__(self, n_qubits: int, term_ptr, op_idx, op_code, coef, check_hermitian: bool = False,
                 force_complex: bool = False, ladder_ints: bool = True, trim_tol: float = 0.0,
                 order_by_mask: bool = False, order_by_parts=None):
        # fermionic operators order their groups by the alpha / beta halves they flip (unless
        # another order is asked for): blocks of rows sharing a beta string reject them in bulk
        if order_by_parts is None:
            order_by_parts = self.fermionic and not order_by_mask
        tp = np.ascontiguousarray(term_ptr, dtype=np.int64)
        oi = np.ascontiguousarray(op_idx, dtype=np.int32)
        oc = np.ascontiguousarray(op_code, dtype=np.uint8)
        c = np.asarray(coef, dtype=np.complex128)
        cr = np.ascontiguousarray(np.stack([c.real, c.imag], axis=1)).astype(np.float64)
        flags = (OP_FERMIONIC if self.fermionic else 0) | (OP_CHECK_HERMITIAN if check_hermitian else 0) | \
                (OP_FORCE_COMPLEX if force_complex else 0) | (0 if ladder_ints else OP_NO_LADDER_INT) | \
                (OP_ORDER_BY_MASK if order_by_mask else 0) | (OP_ORDER_BY_PARTS if order_by_parts else 0)
        h = ctypes.c_void_p()
        _check(lib().qsd_op_compile(int(n_qubits), tp.shape[0] - 1, _ptr(tp), _ptr(oi), _ptr(oc), _ptr(cr), flags,
                                    float(trim_tol), ctypes.byref(h)))
        self._h = h
        self.n_qubits = int(n_qubits)
        T, nl, G, cx, nq = (ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32())
        _check(lib().qsd_op_info(h, ctypes.byref(T), ctypes.byref(nl), ctypes.byref(G), ctypes.byref(cx),
                                 ctypes.byref(nq)))
        self.n_terms, self.n_letters, self.n_groups, self.is_complex = T.value, nl.value, G.value, bool(cx.value)

    @classmethod
    def from_termlist(cls, tl, **kw):
        return cls(tl.n_qubits, tl.term_ptr, tl.op_idx, tl.op_code, tl.coef, **kw)

    @property
    def handle(self):
        return self._h

    def export(self):
        """Compiled terms: ``(term_ptr, op_idx, op_code, coef, group_ptr, group_ladder)``."""
        tp = np.zeros(self.n_terms + 1, dtype=np.int64)
        oi = np.zeros(max(1, self.n_letters), dtype=np.int32)
        oc = np.zeros(max(1, self.n_letters), dtype=np.uint8)
        cr = np.zeros((max(1, self.n_terms), 2), dtype=np.float64)
        gp = np.zeros(self.n_groups + 1, dtype=np.int64)
        gl = np.zeros(self.n_groups, dtype=np.int32)
        _check(lib().qsd_op_export(self._h, _ptr(tp), _ptr(oi), _ptr(oc), _ptr(cr), _ptr(gp), _ptr(gl)))
        return tp, oi[: self.n_letters], oc[: self.n_letters], (cr[:, 0] + 1j * cr[:, 1])[: self.n_terms], gp, gl

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.qsd_op_destroy(h)
            self._h = None


class QubitOperator(_Operator):
    """Sum of words over the extended alphabet (Methods, Qubit Hamiltonians)."""

    fermionic = False


class FermionicOperator(_Operator):
    """Sum of products of f / f^dagger, compiled through the extended JW transform."""

    fermionic = True


def operator_from_termlist(tl, **kw):
    return (FermionicOperator if tl.fermionic else QubitOperator).from_termlist(tl, **kw)


class SubspaceHamiltonian:
    """Operator restricted to a subspace (Methods, Matrix evaluation)."""

    def __init__(self, subspace: Subspace, op: _Operator, stream=None, allocator="default"):
        self.subspace, self.op = subspace, op  # kept alive: the handle references both
        h = ctypes.c_void_p()
        self._allocator = _resolve_allocator(allocator)
        _check(lib().qsd_ham_create(subspace.handle, op.handle, 0, _alloc_arg(self._allocator), _stream(stream),
                                    ctypes.byref(h)))
        self._h = h
        self.N = subspace.N
        self.is_complex = op.is_complex
        self.shape = (self.N, self.N)

    @property
    def handle(self):
        return self._h

    def diagonal(self, stream=None):
        import torch

        d = torch.empty(self.N, dtype=torch.float64, device="cuda")
        _check(lib().qsd_ham_diagonal(self._h, _ptr(d), _stream(stream)))
        return d

    @staticmethod
    def _dtype_code(t):
        import torch

        return {torch.float64: F64, torch.float32: F32, torch.complex128: C128, torch.complex64: C64}[t.dtype]

    def diag_splitting(self, stream=None):
        """``(lowest diagonal element, smallest diagonal splitting)`` over the subspace."""
        lo, sp_ = ctypes.c_double(), ctypes.c_double()
        _check(lib().qsd_ham_diag_splitting(self._h, ctypes.byref(lo), ctypes.byref(sp_), _stream(stream)))
        return lo.value, sp_.value

    def work_counts(self, stream=None):
        """``(probes, hits)`` of one SpMV."""
        p, h = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().qsd_ham_work_counts(self._h, ctypes.byref(p), ctypes.byref(h), _stream(stream)))
        return p.value, h.value

    @property
    def schedule(self) -> int:
        v = ctypes.c_uint32()
        _check(lib().qsd_ham_get_schedule(self._h, ctypes.byref(v)))
        return v.value

    @schedule.setter
    def schedule(self, value: int):
        _check(lib().qsd_ham_set_schedule(self._h, int(value)))

    def autotune(self, nvec: int = 1, dtype=None, reps: int = 3, schedule: bool = True, load: bool = True,
                 split: bool = False, stream=None) -> dict:
        """Times the SpMV under every candidate schedule, hash load and (with ``split``) hash
        family and keeps the fastest (the subspace's table is rebuilt when ``load`` or ``split``)."""
        import torch

        dtype = dtype or (torch.complex128 if self.is_complex else torch.float64)
        code = {torch.float64: F64, torch.float32: F32, torch.complex128: C128, torch.complex64: C64}[dtype]
        flags = (TUNE_SCHEDULE if schedule else 0) | (TUNE_LOAD if load else 0) | (TUNE_SPLIT if split else 0)
        r = TuneResult()
        _check(lib().qsd_ham_autotune(self._h, nvec, code, reps, flags, ctypes.byref(r), _stream(stream)))
        self.subspace._refresh()
        return r.as_dict()

    def matvec(self, x, out=None, stream=None):
        """``H @ x`` for ``x`` of shape ``[N]`` or ``[N][nvec]`` (row-major, interleaved vectors)."""
        import torch

        vec = x.dim() == 1
        X = x.reshape(self.N, -1)
        if X.stride(1) != 1:
            X = X.contiguous()
        nvec = X.shape[1]
        Y = torch.empty_like(X) if out is None else out.reshape(self.N, -1)
        _check(lib().qsd_matvec(self._h, nvec, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0), self._dtype_code(X),
                                _stream(stream)))
        return Y.reshape(-1) if vec else Y

    def ramps(self, s0, E: float, tau: float, max_depth: int = 32, max_frontier: int = 1 << 22, stream=None):
        """RAMPS restricted to this subspace (Supplement, Algorithm S1): ``(mask, info)`` with
        ``mask`` a device uint8 [N] tensor marking S_0 and the selected strings."""
        import torch

        idx = np.ascontiguousarray(np.asarray(s0, dtype=np.int64).reshape(-1))
        mask = torch.empty(self.N, dtype=torch.uint8, device="cuda")
        info = RampsInfo()
        n = ctypes.c_int64()
        _check(lib().qsd_ramps(self._h, _ptr(idx), idx.size, float(E), float(tau), int(max_depth), int(max_frontier),
                               _ptr(mask), ctypes.byref(n), ctypes.byref(info), _stream(stream)))
        return mask, info.as_dict()

    def matvec_raw(self, nvec, x_ptr, ldx, y_ptr, ldy, dtype, stream=None):
        _check(lib().qsd_matvec(self._h, nvec, ctypes.c_void_p(x_ptr), ldx, ctypes.c_void_p(y_ptr), ldy, dtype,
                                _stream(stream)))

    def to_csr(self, index_type: int = INDEX_I64, dtype=None, stream=None):
        """Two-pass CSR: ``(indptr int64, indices, data)`` device tensors."""
        import torch

        if dtype is None:
            dtype = torch.complex128 if self.is_complex else torch.float64
        code = {torch.float64: F64, torch.float32: F32, torch.complex128: C128, torch.complex64: C64}[dtype]
        indptr = torch.empty(self.N + 1, dtype=torch.int64, device="cuda")
        nnz = ctypes.c_int64()
        st = _stream(stream)
        _check(lib().qsd_csr_build(self._h, _ptr(indptr), None, None, index_type, code, ctypes.byref(nnz), st))
        idx = torch.empty(max(1, nnz.value), dtype=torch.int32 if index_type == INDEX_I32 else torch.int64,
                          device="cuda")
        data = torch.empty(max(1, nnz.value), dtype=dtype, device="cuda")
        _check(lib().qsd_csr_build(self._h, _ptr(indptr), _ptr(idx), _ptr(data), index_type, code, ctypes.byref(nnz),
                                   st))
        return indptr, idx[: nnz.value], data[: nnz.value]

    def lanczos(self, max_iter=300, tol=1e-10, v0="uniform", seed=0, spmv_dtype="f64", check_every=5,
                want_vector=False, use_graph=False, v0_vector=None, stream=None, raise_on_nonconv=True, block=1):
        """Lowest eigenvalue by GPU Lanczos: ``(energy, vector or None, info dict)``.

        ``block`` 4, 8 or 16 runs block Lanczos (``max_iter`` then counts block steps)."""
        return _lanczos(lib().qsd_lanczos, lib().qsd_block_lanczos, self._h, self.N, max_iter, tol, v0, seed,
                        spmv_dtype, check_every, want_vector, use_graph, v0_vector, stream, raise_on_nonconv, block,
                        self.is_complex)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.qsd_ham_destroy(h)
            self._h = None


def trimmed_hamiltonian(ham: "SubspaceHamiltonian", tl, tol: float, stream=None):
    """The Hamiltonian of term list ``tl`` on ``ham``'s subspace with the groups whose bound is
    below ``tol`` times the subspace's smallest diagonal splitting removed (Results, CH4-dimer
    runs): ``(trimmed SubspaceHamiltonian, absolute threshold)``."""
    _, split = ham.diag_splitting(stream)
    op = operator_from_termlist(tl, trim_tol=tol * split)
    return SubspaceHamiltonian(ham.subspace, op, stream), tol * split


def _lanczos(single, blockfn, handle, N, max_iter, tol, v0, seed, spmv_dtype, check_every, want_vector, use_graph,
             v0_vector, stream, raise_on_nonconv, block, is_complex=False):
    import torch

    o = LanczosOpts()
    lib().qsd_lanczos_default_opts(ctypes.byref(o))
    o.max_iter, o.tol, o.seed, o.check_every = max_iter, tol, seed, check_every
    o.v0_mode = {"uniform": V0_UNIFORM, "min_diag": V0_MIN_DIAG, "random": V0_RANDOM, "user": V0_USER}[v0]
    o.spmv_dtype = {"f64": F64, "f32": F32}[spmv_dtype]
    o.want_vector, o.use_graph = int(want_vector), int(use_graph)
    vec = None
    if want_vector or v0 == "user":
        vec = torch.empty(N, dtype=torch.complex128 if is_complex else torch.float64, device="cuda")
        if v0 == "user":
            vec.copy_(v0_vector)
    e = ctypes.c_double()
    info = LanczosInfo()
    if block == 1:
        rc = single(handle, ctypes.byref(o), ctypes.byref(e), _ptr(vec), ctypes.byref(info), _stream(stream))
    else:
        rc = blockfn(handle, int(block), ctypes.byref(o), ctypes.byref(e), _ptr(vec), ctypes.byref(info),
                     _stream(stream))
    if rc != QSD_OK and not (rc == -6 and not raise_on_nonconv):
        _check(rc)
    return e.value, (vec if want_vector else None), info.as_dict()


class CsrMatrix:
    """The operator's CSR matrix kept on the device (``qsd_csr_*``): SpMV and Lanczos on it."""

    def __init__(self, ham: "SubspaceHamiltonian", index_type: int = INDEX_I32, dtype=None,
                 lower_mirror: bool = False, stream=None, allocator="default"):
        import torch

        if dtype is None:
            dtype = torch.complex128 if ham.is_complex else torch.float64
        self.dtype = dtype
        code = {torch.float64: F64, torch.float32: F32, torch.complex128: C128, torch.complex64: C64}[dtype]
        h = ctypes.c_void_p()
        self._allocator = _resolve_allocator(allocator)
        _check(lib().qsd_csr_create(ham.handle, index_type, code, CSR_LOWER_MIRROR if lower_mirror else 0,
                                    _alloc_arg(self._allocator), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.index_type = index_type
        N, nnz, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().qsd_csr_info(h, ctypes.byref(N), ctypes.byref(nnz), ctypes.byref(b)))
        self.N, self.nnz, self.bytes = N.value, nnz.value, b.value
        self.is_complex = ham.is_complex

    @property
    def handle(self):
        return self._h

    def export(self, stream=None):
        """``(indptr int64, indices, data)`` device tensors (copies)."""
        import torch

        ip = torch.empty(self.N + 1, dtype=torch.int64, device="cuda")
        ix = torch.empty(max(1, self.nnz), dtype=torch.int32 if self.index_type == INDEX_I32 else torch.int64,
                         device="cuda")
        dv = torch.empty(max(1, self.nnz), dtype=self.dtype, device="cuda")
        _check(lib().qsd_csr_export(self._h, _ptr(ip), _ptr(ix), _ptr(dv), _stream(stream)))
        return ip, ix[: self.nnz], dv[: self.nnz]

    def matvec(self, x, out=None, stream=None):
        vec = x.dim() == 1
        X = x.reshape(self.N, -1)
        if X.stride(1) != 1:
            X = X.contiguous()
        nvec = X.shape[1]
        Y = torch_empty_like(X) if out is None else out.reshape(self.N, -1)
        _check(lib().qsd_csr_matvec(self._h, nvec, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0),
                                    SubspaceHamiltonian._dtype_code(X), _stream(stream)))
        return Y.reshape(-1) if vec else Y

    def lanczos(self, max_iter=300, tol=1e-10, v0="uniform", seed=0, spmv_dtype=None, check_every=5,
                want_vector=False, use_graph=False, v0_vector=None, stream=None, raise_on_nonconv=True, block=1):
        """Lanczos on the stored matrix (see ``SubspaceHamiltonian.lanczos``)."""
        import torch

        if spmv_dtype is None:
            spmv_dtype = "f32" if self.dtype in (torch.float32, torch.complex64) else "f64"
        return _lanczos(lib().qsd_csr_lanczos, lib().qsd_csr_block_lanczos, self._h, self.N, max_iter, tol, v0, seed,
                        spmv_dtype, check_every, want_vector, use_graph, v0_vector, stream, raise_on_nonconv, block,
                        self.is_complex)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.qsd_csr_destroy(h)
            self._h = None


def torch_empty_like(x):
    import torch

    return torch.empty_like(x)


def _matvec_batched(entry, hams, xs, ys, stream):
    import torch

    n = len(hams)
    if ys is None:
        ys = [torch.empty_like(x) for x in xs]
    if n == 0:
        return ys
    code = SubspaceHamiltonian._dtype_code(xs[0])
    for h, x, y in zip(hams, xs, ys):
        if not (x.is_contiguous() and y.is_contiguous()) or x.shape[0] != h.N or y.shape != x.shape:
            raise ValueError("vectors must be contiguous [N] or [N][nvec] tensors matching their operator")
    H = (ctypes.c_void_p * n)(*[h.handle.value for h in hams])
    X = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    Y = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ys])
    nv = np.array([1 if x.dim() == 1 else x.shape[1] for x in xs], dtype=np.int32)
    _check(entry(n, ctypes.cast(H, ctypes.c_void_p), ctypes.cast(X, ctypes.c_void_p), ctypes.cast(Y, ctypes.c_void_p),
                 _ptr(nv), code, _stream(stream)))
    return ys


def matvec_batched(hams, xs, ys=None, stream=None):
    """``ys[i] = hams[i] @ xs[i]`` for every request in one launch per key width
    (``qsd_matvec_batched``); vectors are ``[N]`` or ``[N][nvec]`` contiguous device tensors of
    one dtype."""
    return _matvec_batched(lib().qsd_matvec_batched, hams, xs, ys, stream)


def matvec_batched_noalloc(hams, xs, ys, stream=None):
    """``matvec_batched`` through ``qsd_matvec_batched_noalloc``: the library allocates nothing
    (its tables live in a fixed per-GPU device array), so ``ys`` must be given.  At most
    ``NOALLOC_MAX_REQUESTS`` request chunks and ``NOALLOC_MAX_TILES`` row tiles of 256 rows;
    calls that overlap on one GPU race on the shared array."""
    if ys is None:
        raise ValueError("matvec_batched_noalloc writes into caller-provided ys")
    return _matvec_batched(lib().qsd_matvec_batched_noalloc, hams, xs, ys, stream)


class LanczosBatch:
    """Continuous-batching Lanczos: many ground-state solves advance one iteration per step
    with one batched SpMV launch (``qsd_batch_*``)."""

    RUNNING, CONVERGED, LIMIT = 1, 2, 3

    def __init__(self, max_requests: int, max_iter: int = 300, spmv_dtype: str = "f64", allocator="default"):
        self.max_requests, self.max_iter = int(max_requests), int(max_iter)
        self.dtype = {"f64": F64, "f32": F32}[spmv_dtype]
        h = ctypes.c_void_p()
        self._allocator = _resolve_allocator(allocator)
        _check(lib().qsd_batch_create(self.max_requests, self.max_iter, self.dtype, _alloc_arg(self._allocator),
                                      ctypes.byref(h)))
        self._h = h
        self._hams = {}

    def footprint(self, ham) -> int:
        """Workspace bytes of a request on ``ham`` (a SubspaceHamiltonian or a CsrMatrix)."""
        b = ctypes.c_int64()
        _check(lib().qsd_batch_footprint_rows(int(ham.N), self.max_iter, self.dtype, ctypes.byref(b)))
        return b.value

    def add(self, ham: "SubspaceHamiltonian", v0: str = "uniform", seed: int = 0, tol: float = 1e-10,
            workspace=None, stream=None):
        """Start a solve; ``workspace`` (a device tensor of at least ``footprint`` bytes) is kept
        by the batch until the slot is removed; ``None`` lets the library allocate."""
        mode = {"uniform": V0_UNIFORM, "min_diag": V0_MIN_DIAG, "random": V0_RANDOM}[v0]
        slot = ctypes.c_int32()
        nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
        add = lib().qsd_batch_add_csr if isinstance(ham, CsrMatrix) else lib().qsd_batch_add
        _check(add(self._h, ham.handle, mode, seed, tol, _ptr(workspace), nbytes, ctypes.byref(slot), _stream(stream)))
        self._hams[slot.value] = (ham, workspace)  # both stay alive while the request runs
        return slot.value

    def step(self, iterations: int = 1, stream=None):
        _check(lib().qsd_batch_step(self._h, int(iterations), _stream(stream)))

    def poll(self, stream=None):
        n = self.max_requests
        st = np.zeros(n, dtype=np.int32)
        e = np.zeros(n, dtype=np.float64)
        it = np.zeros(n, dtype=np.int32)
        rr = np.zeros(n, dtype=np.float64)
        _check(lib().qsd_batch_poll(self._h, _ptr(st), _ptr(e), _ptr(it), _ptr(rr), _stream(stream)))
        return st, e, it, rr

    def remove(self, slot: int):
        _check(lib().qsd_batch_remove(self._h, int(slot)))
        self._hams.pop(int(slot), None)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.qsd_batch_destroy(h)
            self._h = None
