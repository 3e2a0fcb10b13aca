"""GPU parity of the product map: alpha x beta product subspaces (Results, fermionic examples)
whose SpMV takes each column's index from the ranks of its two parts instead of the hash table.

The map is found when the subspace is built; the results must equal the oracle's bit for bit
(dyadic data) and the hash-table path's (QSD_SCHED_HASH_LOOKUP) under every schedule.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import rowwise as orw
from oracle import subspace as osub

from _util import c2_keys, c3_parts, dyadic, dyadic_vector, say

torch = pytest.importorskip("torch")
qsd = pytest.importorskip("paper_2603_18731_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qsd.lib()


def _all_schedules(H, x):
    """Output of every schedule, with and without the hash-table lookup, each written into a
    NaN-filled buffer (a row that no lane writes stays NaN and fails the comparison)."""
    outs = []
    for sched in range(2 * (qsd.SCHED_ALL + 1)):
        H.schedule = sched
        y = torch.full_like(x, float("nan"))
        H.matvec(x, out=y)
        outs.append((sched, y))
    torch.cuda.synchronize()
    return outs


def test_product_detected():
    ops, keys = c3_parts(37, 29)
    sub = qsd.Subspace(keys, ops.n_qubits)
    assert sub.N == 37 * 29
    split, _, product = sub.hash_info()
    assert split == 16 and product
    idx = sub.lookup(keys)
    # one string missing: not a product, no part filters
    sub2 = qsd.Subspace(np.ascontiguousarray(keys[1:]), ops.n_qubits)
    assert sub2.hash_info()[0] == 0 and not sub2.hash_info()[2]
    # the same strings split elsewhere, or not at all: no map; split at 16 again: the map
    for load, split, want in ((0.125, 0, False), (0.25, 5, False), (0.5, 16, True), (0.03125, 16, True)):
        sub.rehash(load, split)
        assert sub.hash_info()[0] == split and sub.hash_info()[2] == want
        assert torch.equal(sub.lookup(keys), idx)
    # a sample that is not a product (36 qubits, one key word, halves of 18)
    assert not qsd.Subspace(c2_keys(5_000), 36).hash_info()[2]
    # a single alpha string (the map's low part count is 1) and a single beta string
    w = wl.c3_molecular(1, 40)
    assert qsd.Subspace(w.keys, w.ops.n_qubits).hash_info()[2]
    w = wl.c3_molecular(40, 1)
    assert qsd.Subspace(w.keys, w.ops.n_qubits).hash_info()[2]


ORDERS = {"parts": {}, "weight": {"order_by_parts": False}, "mask": {"order_by_mask": True}}


@pytest.mark.parametrize("na,nb,order", [(37, 29, "parts"), (70, 70, "parts"), (70, 70, "weight"), (70, 70, "mask"),
                                         (128, 3, "parts"), (1, 200, "parts"), (300, 1, "weight"),
                                         (600, 7, "parts"), (513, 3, "weight")])
def test_product_matvec_exact(na, nb, order):
    """Dyadic coefficients and vectors: every schedule, with the map and through the table,
    under each group order, equals the oracle bit for bit (one vector, three interleaved
    vectors, and FP32 elements and vectors with FP64 accumulation, whose result is the exact
    value rounded once).  With 512 or more alpha strings the map kernel's tiles follow the
    product's blocks of rows (600 = 2 x 256 + 88, 513 = 2 x 256 + 1)."""
    ops, keys = c3_parts(na, nb) if na > 1 and nb > 1 else (None, None)
    if ops is None:
        w = wl.c3_molecular(na, nb)
        ops, keys = w.ops, w.keys
    tl = dyadic(ops)
    say("product matvec", na, nb, order)
    sub = qsd.Subspace(keys, tl.n_qubits)
    assert sub.hash_info()[2]
    H = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(tl, **ORDERS[order]))
    ck = osub.canonical_keys(keys)
    rng = np.random.default_rng(na * 1000 + nb)
    X = dyadic_vector(rng, sub.N, nvec=3)
    Y_o = orw.matvec_c(ck, tl, X).real
    for sched, y in _all_schedules(H, torch.from_numpy(X).cuda()):
        np.testing.assert_array_equal(y.cpu().numpy(), Y_o, err_msg="schedule %d" % sched)
    x1 = np.ascontiguousarray(X[:, 0])
    for sched, y in _all_schedules(H, torch.from_numpy(x1).cuda()):
        np.testing.assert_array_equal(y.cpu().numpy(), Y_o[:, 0], err_msg="schedule %d" % sched)
    tl8 = dyadic(ops, bits=8)
    H8 = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(tl8, **ORDERS[order]))
    X6 = dyadic_vector(rng, sub.N, bits=6, nvec=2)
    Y8 = orw.matvec_c(ck, tl8, X6).real.astype(np.float32)
    for sched, y in _all_schedules(H8, torch.from_numpy(X6.astype(np.float32)).cuda()):
        np.testing.assert_array_equal(y.cpu().numpy(), Y8, err_msg="fp32 schedule %d" % sched)


def test_product_wide_spmm_and_solver():
    """8 and 16 interleaved vectors under the map equal the oracle (dyadic), and a Lanczos solve
    gives bitwise the same energy with the map and through the table."""
    ops, keys = c3_parts(60, 45)
    tl = dyadic(ops)
    sub = qsd.Subspace(keys, tl.n_qubits)
    H = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(tl))
    ck = osub.canonical_keys(keys)
    rng = np.random.default_rng(12)
    for nv in (8, 16):
        X = dyadic_vector(rng, sub.N, nvec=nv)
        np.testing.assert_array_equal(H.matvec(torch.from_numpy(X).cuda()).cpu().numpy(),
                                      orw.matvec_c(ck, tl, X).real)
    Hr = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(ops))
    Hr.schedule = qsd.SCHED_FILTER_FIRST | qsd.SCHED_XCD_REMAP
    e_map, _, _ = Hr.lanczos(tol=1e-10, max_iter=200)
    Hr.schedule |= qsd.SCHED_HASH_LOOKUP
    e_tab, _, _ = Hr.lanczos(tol=1e-10, max_iter=200)
    say("energies", e_map, e_tab)
    assert e_map == e_tab


def test_product_group_over_65535_terms():
    """A group too long for 16-bit range pointers (X0 X1 times 70 000 distinct Z strings, so no
    ladder integer) beside ladder, projector and diagonal terms: the product-map kernel keeps such
    a group's term count split over its first two range pointers; every schedule, with the map
    and through the table, equals the oracle bit for bit (dyadic data)."""
    _, keys = c3_parts(40, 30)
    rng = np.random.default_rng(65536)
    masks = np.unique(rng.integers(1, 1 << 30, size=72_000, dtype=np.int64))[:70_000] << 2
    assert masks.shape[0] == 70_000
    terms = []
    for m in masks.tolist():
        word = [(0, 3), (1, 3)] + [(q, 0) for q in range(2, 32) if (m >> q) & 1]
        terms.append((float(rng.integers(-512, 512) or 1) / 1024.0, word))
    terms += [(0.25, [(5, 6), (7, 5)]), (0.25, [(7, 6), (5, 5)]), (-0.5, [(18, 6), (20, 5), (3, 2)]),
              (0.75, [(2, 3), (17, 3)]), (0.125, [(4, 0), (21, 0)]), (-1.0, [])]
    tl = wl.TermList.from_terms(32, terms)
    say("long group", len(terms), "terms")
    sub = qsd.Subspace(keys, 32)
    assert sub.hash_info()[2]
    op = qsd.operator_from_termlist(tl)
    gptr, glad = op.export()[4:]
    big = int(np.argmax(np.diff(gptr)))
    assert np.diff(gptr)[big] == 70_000 and glad[big] == 0
    H = qsd.SubspaceHamiltonian(sub, op)
    ck = osub.canonical_keys(keys)
    x = dyadic_vector(rng, sub.N)
    y_o = orw.matvec_c(ck, tl, x).real
    assert np.count_nonzero(y_o) > sub.N // 2
    for sched, y in _all_schedules(H, torch.from_numpy(x).cuda()):
        np.testing.assert_array_equal(y.cpu().numpy(), y_o, err_msg="schedule %d" % sched)
