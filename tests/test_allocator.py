"""The caller's device allocator (qsd_allocator): every byte a handle or a call takes comes from
it and goes back to it; a failing allocation is reported as OUT_OF_MEMORY after everything
taken so far has been returned.

The CPU tests reach only paths that fail at their first allocation (no device work is ever
enqueued); the GPU tests fail the k-th allocation of each creating call for every k."""
import ctypes

import numpy as np
import pytest

import workloads as wl

from _util import c3_parts, say

qsd = pytest.importorskip("paper_2603_18731_amd")

ERR_OOM = -2


class Counting:
    """Allocator that records live blocks and fails its `fail_at`-th call (1-based); blocks come
    from `inner(nbytes, stream)` (None: fail every call)."""

    def __init__(self, inner=None, release=None, fail_at=None):
        self.inner, self.release, self.fail_at = inner, release, fail_at
        self.calls, self.live = 0, {}
        self.struct = qsd.Allocator(None, qsd.ALLOC_FN(self._alloc), qsd.FREE_FN(self._free))

    def _alloc(self, ctx, nbytes, stream):
        self.calls += 1
        if self.inner is None or self.calls == self.fail_at:
            return None
        p = self.inner(int(nbytes), stream)
        if p:
            self.live[int(p)] = int(nbytes)
        return p

    def _free(self, ctx, ptr, stream):
        assert int(ptr) in self.live, "free of a block this allocator did not hand out"
        del self.live[int(ptr)]
        if self.release:
            self.release(int(ptr))


def _lib_or_skip():
    import os

    if not os.path.exists(qsd.LIB_PATH):
        pytest.skip("libqsd.so not built")
    return qsd.lib()


def test_null_allocator_fails_cleanly():
    """An allocator that returns NULL: creating calls fail with OUT_OF_MEMORY before any device
    work, and nothing is left allocated."""
    L = _lib_or_skip()
    a = Counting()
    dummy = ctypes.c_uint64(0)
    h = ctypes.c_void_p()
    rc = L.qsd_subspace_build(ctypes.byref(dummy), 1, 8, 0, 0.0, ctypes.byref(a.struct), None, ctypes.byref(h))
    assert rc == ERR_OOM and not h.value and a.calls == 1 and not a.live
    assert b"allocation" in L.qsd_last_error()
    rc = L.qsd_batch_create(4, 50, qsd.F64, ctypes.byref(a.struct), ctypes.byref(h))
    assert rc == ERR_OOM and not h.value and a.calls == 2 and not a.live


# ------------------------------------------------------------------------------ GPU

def _torch_counting(fail_at=None):
    import torch

    return Counting(lambda n, s: torch.cuda.caching_allocator_alloc(n, stream=int(s or 0)),
                    torch.cuda.caching_allocator_delete, fail_at)


@pytest.mark.gpu
def test_every_allocation_failure_is_clean():
    """Fail the k-th allocation of subspace build, rehash with part filters, operator bind, CSR
    build, stored CSR, Lanczos and block Lanczos, for every k: OUT_OF_MEMORY, and all blocks
    taken so far are returned.  With no failure every block is returned at destruction."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ops, keys = c3_parts(30, 30)
    op = qsd.operator_from_termlist(ops)

    def run(a):
        """Energies, or the error code of the first failing call (the handles created so far
        are released when this frame ends)."""
        try:
            sub = qsd.Subspace(keys, ops.n_qubits, allocator=a.struct)
            sub.rehash(0.25, 16)
            H = qsd.SubspaceHamiltonian(sub, op, allocator=a.struct)
            H.to_csr()
            A = qsd.CsrMatrix(H, lower_mirror=True, allocator=a.struct)
            return (H.lanczos(tol=1e-10)[0], A.lanczos(tol=1e-10)[0],
                    H.lanczos(tol=1e-9, block=4, max_iter=40)[0])
        except qsd.QsdError as exc:
            return exc.code

    import gc

    ok = _torch_counting()
    e = run(ok)
    gc.collect()
    torch.cuda.synchronize()
    say("allocations", ok.calls, "energies", e)
    assert not ok.live and ok.calls > 10
    assert abs(e[0] - e[1]) < 1e-10 * abs(e[0]) and abs(e[0] - e[2]) < 1e-9 * abs(e[0])
    for k in range(1, ok.calls + 1):
        a = _torch_counting(fail_at=k)
        assert run(a) == ERR_OOM, k
        gc.collect()
        torch.cuda.synchronize()
        assert not a.live, (k, a.live)


@pytest.mark.gpu
def test_torch_allocator_accounts_the_library():
    """With the default (PyTorch) allocator the library's device memory shows in
    torch.cuda.memory_allocated and is returned at destruction."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    w = wl.c2_xxz6x6(50_000)
    sub = qsd.Subspace(w.keys, w.ops.n_qubits)
    H = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(w.ops))
    held = torch.cuda.memory_allocated() - before
    # keys, hashes, slot order, table (capacity slots) and the diagonal at least
    assert held >= sub.capacity * 8 + sub.N * (8 + 8 + 8)
    del H, sub
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
