"""Ground energies of the large workloads on the GPU against the CPU oracle's.

``tests/golden/energies.json`` holds the lowest eigenvalue of each workload's H_S as found by
two CPU eigensolvers (the oracle's Lanczos and ARPACK) on the oracle's term-by-term matrix
(``tests/golden/make_energies.py``).  The GPU solvers (Lanczos on the matrix-free SpMV, on the
stored CSR, block Lanczos) must agree within 1e-10 relative in FP64; the FP32-SpMV solves (FP64
orthogonalization and recurrence) are reported against the same FP64 reference and bounded.
"""
import json
import os

import numpy as np
import pytest

import workloads as wl

from _util import say

torch = pytest.importorskip("torch")
qsd = pytest.importorskip("paper_2603_18731_amd")

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "energies.json")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qsd.lib()


def _golden(name):
    with open(GOLDEN) as f:
        return json.load(f)[name]["energy"]


def _rel(a, b):
    return abs(a - b) / abs(b)


def _ham(w, **kw):
    sub = qsd.Subspace(w.keys, w.ops.n_qubits)
    return sub, qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(w.ops, **kw))


def test_energy_xxz6x6_full():
    e_ref = _golden("xxz6x6_w18_1048576")
    sub, H = _ham(wl.c2_xxz6x6())
    sub.rehash(1 / 32)
    H.schedule = qsd.SCHED_ALL
    e, _, info = H.lanczos(tol=1e-12, max_iter=300)
    say("xxz6x6 full", e, e_ref, info["iterations"])
    assert _rel(e, e_ref) < 1e-10
    e32, _, _ = H.lanczos(tol=1e-8, max_iter=300, spmv_dtype="f32")
    say("xxz6x6 full fp32 rel err", _rel(e32, e_ref))
    assert _rel(e32, e_ref) < 1e-6


def test_energy_fermi16_300x300():
    """The reduced fermionic product subspace (300 x 300 determinants), matrix-free with and
    without part filters, from the stored CSR, and block Lanczos."""
    e_ref = _golden("fermi16_300x300")
    sub, H = _ham(wl.c3_molecular(300, 300))
    res = {}
    e, _, info = H.lanczos(tol=1e-12, max_iter=300)
    res["matrix-free"] = e
    sub.rehash(1 / 32, 16)
    H.schedule = qsd.SCHED_FILTER_FIRST
    res["part filters"] = H.lanczos(tol=1e-12, max_iter=300)[0]
    res["block 8"] = H.lanczos(tol=1e-11, max_iter=80, block=8)[0]
    res["csr"] = qsd.CsrMatrix(H, lower_mirror=True).lanczos(tol=1e-12, max_iter=300)[0]
    say("fermi16 300x300", res, e_ref)
    for k, v in res.items():
        assert _rel(v, e_ref) < 1e-10, k
    e32, _, _ = H.lanczos(tol=1e-8, max_iter=300, spmv_dtype="f32")
    say("fermi16 300x300 fp32 rel err", _rel(e32, e_ref))
    assert _rel(e32, e_ref) < 1e-6


def test_energy_heavyhex200_full():
    """The 5M-string heavy-hex workload: single-vector and block-8 Lanczos (FP64 and FP32 SpMM)."""
    e_ref = _golden("heavyhex200_5000000")
    sub, H = _ham(wl.c4_heavy_hex())
    sub.rehash(1 / 32)
    H.schedule = qsd.SCHED_ALL
    e, _, info = H.lanczos(tol=1e-12, max_iter=300)
    eb, _, infob = H.lanczos(tol=1e-11, max_iter=80, block=8)
    eb32, _, _ = H.lanczos(tol=1e-8, max_iter=80, block=8, spmv_dtype="f32")
    say("heavyhex full", e, eb, eb32, e_ref, info["iterations"], infob["iterations"])
    assert _rel(e, e_ref) < 1e-10
    assert _rel(eb, e_ref) < 1e-10
    assert _rel(eb32, e_ref) < 1e-6
