"""SpMV schedules and the autotuner: every schedule gives bitwise the same output (each row is
evaluated by one lane in the same order whatever workgroup runs it), and the autotuner keeps
one of them."""
import numpy as np
import pytest

import workloads as wl

from _util import c2_keys, c3_parts, heavy_hex_small, say

torch = pytest.importorskip("torch")
qsd = pytest.importorskip("paper_2603_18731_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qsd.lib()


def _ham(keys, tl):
    return qsd.SubspaceHamiltonian(qsd.Subspace(keys, tl.n_qubits), qsd.operator_from_termlist(tl))


def _case(case):
    if case == "xxz":
        return _ham(c2_keys(50_000), wl.xxz_grid_6x6())
    if case == "fermi":
        ops, keys = c3_parts(90, 90)
        return _ham(keys, ops)
    if case == "complex":
        rng = np.random.default_rng(21)
        n = 14
        terms = []
        for _ in range(60):
            m = int(rng.integers(1, 4))
            qs = rng.choice(n, size=m, replace=False)
            word = [(int(q), int(rng.integers(0, 7))) for q in qs]
            c = complex(rng.normal(), rng.normal())
            terms.append((c, word))
            terms.append((c.conjugate(), [(q, {5: 6, 6: 5}.get(k, k)) for q, k in word]))
        tl = wl.TermList.from_terms(n, terms)
        from oracle import subspace as osub

        keys = osub.ints_to_keys(sorted(rng.choice(1 << n, size=5000, replace=False).tolist()), 1)
        return _ham(keys, tl)
    if case == "diagonal":
        # no off-diagonal groups: the slot-order schedules write y from the diagonal pass alone
        n = 12
        tl = wl.TermList.from_terms(n, [(-1.0 - 0.25 * i, [(i, 0), ((i + 1) % n, 0)]) for i in range(n)]
                                    + [(0.5, [(0, 2)])])
        return _ham(wl.c1_tfim12().keys[::3].copy(), tl)
    tl, keys = heavy_hex_small(30_001)
    return _ham(keys, tl)


def _run_all(H, x):
    """One output per schedule, each written into a NaN-filled buffer (a row no lane writes stays
    NaN and fails the comparison)."""
    outs = []
    for sched in range(qsd.SCHED_ALL + 1):
        H.schedule = sched
        y = torch.full_like(x, float("nan"))
        H.matvec(x, out=y)
        outs.append(y)
    torch.cuda.synchronize()
    return outs


@pytest.mark.parametrize("case", ["xxz", "fermi", "heavyhex", "complex", "diagonal"])
def test_schedules_bitwise(case):
    H = _case(case)
    rng = np.random.default_rng(3)
    if H.is_complex:
        x = torch.from_numpy(rng.standard_normal((H.N, 2)) + 1j * rng.standard_normal((H.N, 2))).cuda()
    else:
        x = torch.from_numpy(rng.standard_normal((H.N, 3))).cuda()
    outs = _run_all(H, x)
    say(case, "N", H.N)
    assert not torch.isnan(outs[0]).any()
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    if case == "diagonal":
        assert torch.equal(outs[0], H.diagonal()[:, None] * x)
    if not H.is_complex:
        # single precision and one vector, through the slot-order lockstep schedule
        x32 = x[:, :1].float().contiguous()
        o32 = _run_all(H, x32)
        for o in o32[1:]:
            assert torch.equal(o, o32[0])
    r = H.autotune(nvec=x.shape[1], dtype=x.dtype, reps=2)
    say(case, "autotune ->", r)
    assert 0 <= r["schedule"] <= qsd.SCHED_ALL and H.schedule == r["schedule"] and r["ms"] > 0
    # (a product subspace keeps its table: the SpMV does not read it)
    assert r["max_load"] in (0.03125, 0.0625, 0.125, 0.25, 0.5) or H.subspace.hash_info()[2]
    assert H.subspace.capacity == r["capacity"]
    assert torch.equal(H.matvec(x), outs[0])  # a rebuilt table gives the same output
    keys_before = H.subspace.keys()
    nq = H.subspace.n_qubits
    # other loads, and part filters (a split at the middle, near the bottom and near the top)
    for load, split in ((0.5, 0), (0.03, 0), (0.25, nq // 2), (0.5, 3), (0.0625, nq - 1)):
        H.subspace.rehash(load, split)
        assert H.subspace.hash_info()[0] == split
        for o in _run_all(H, x):  # the slot order and the group part indices follow the table
            assert torch.equal(o, outs[0])
        assert torch.equal(H.subspace.lookup(keys_before), torch.arange(H.N, device="cuda"))
    r = H.autotune(nvec=x.shape[1], dtype=x.dtype, reps=1, split=True)
    assert r["split"] == H.subspace.hash_info()[0] and torch.equal(H.matvec(x), outs[0])
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        H.subspace.rehash(0.25, nq)
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        H.schedule = 0x80


def test_part_filters_groups_by_mask_exact():
    """The fermionic product subspace with groups ordered by flip mask and part filters split at
    the first beta qubit (exact filters), at a mid-alpha qubit, and none, under every schedule:
    equal to the oracle bit for bit (dyadic data)."""
    from oracle import rowwise as orw
    from oracle import subspace as osub

    from _util import dyadic, dyadic_vector

    ops, keys = c3_parts(90, 90)
    tl = dyadic(ops)
    sub = qsd.Subspace(keys, tl.n_qubits)
    H = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(tl, order_by_mask=True))
    rng = np.random.default_rng(31)
    x = torch.from_numpy(dyadic_vector(rng, H.N, nvec=2)).cuda()
    y_o = orw.matvec_c(osub.canonical_keys(keys), tl, x.cpu().numpy()).real
    for load, split in ((0.125, 16), (0.5, 16), (0.03125, 16), (0.25, 5), (0.25, 0)):
        sub.rehash(load, split)
        assert sub.hash_info()[0] == split
        say("split", split, "capacity", sub.capacity)
        for o in _run_all(H, x):
            np.testing.assert_array_equal(o.cpu().numpy(), y_o)


@pytest.mark.parametrize("case", ["xxz", "heavyhex", "complex"])
def test_solvers_under_slot_order_schedules(case):
    """Lanczos (plain, HIP-graph replay, FP32 SpMV) and block Lanczos give the same energies under
    the slot-order lockstep schedule (two kernels per FP64 SpMV) as under the canonical one."""
    H = _case(case)
    res = {}
    side = torch.cuda.Stream()  # graph capture needs a non-default stream
    for sched in (0, qsd.SCHED_ALL):
        H.schedule = sched
        e, _, info = H.lanczos(tol=1e-10, max_iter=400)
        with torch.cuda.stream(side):
            eg, _, _ = H.lanczos(tol=1e-10, max_iter=400, use_graph=True)
        torch.cuda.synchronize()
        r = [e, eg]
        if not H.is_complex:
            e32, _, _ = H.lanczos(tol=1e-6, max_iter=400, spmv_dtype="f32")
            eb, _, _ = H.lanczos(tol=1e-9, max_iter=60, block=4)
            r += [e32, eb]
        res[sched] = r
        say(case, "schedule", sched, r, info["iterations"])
    for a, b in zip(res[0], res[qsd.SCHED_ALL]):
        assert abs(a - b) <= 1e-9 * abs(a)
    assert res[0][0] == res[0][1]  # graph replay runs the same kernels
    assert res[qsd.SCHED_ALL][0] == res[qsd.SCHED_ALL][1]


@pytest.mark.parametrize("n_rows", [1, 2, 63, 65, 257, 900])
def test_schedules_ragged_sizes(n_rows):
    """Tiny and ragged subspaces (fewer rows than a wave, a workgroup or eight workgroups) under
    every schedule: the same output bitwise, equal to the oracle (dyadic data: exact sums)."""
    from oracle import rowwise as orw
    from oracle import subspace as osub

    from _util import dyadic, dyadic_vector

    rng = np.random.default_rng(100 + n_rows)
    n = 12
    tl = dyadic(wl.xxz_terms(n, [(i, (i + 1) % n) for i in range(n)], 1.0, 0.75))
    # strings of weight 6 (the XXZ sector), so that columns often land in the subspace
    pool = [v for v in range(1 << n) if bin(v).count("1") == 6]
    keys = osub.ints_to_keys(sorted(rng.choice(pool, size=n_rows, replace=False).tolist()), 1)
    H = _ham(keys, tl)
    x = torch.from_numpy(dyadic_vector(rng, H.N, nvec=2)).cuda()
    outs = _run_all(H, x)
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    y_o = orw.matvec_c(osub.canonical_keys(keys), tl, x.cpu().numpy()).real
    np.testing.assert_array_equal(outs[0].cpu().numpy(), y_o)
