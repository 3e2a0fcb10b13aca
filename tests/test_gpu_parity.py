"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle, element by element.

Bit-exact: canonical keys, hash lookups, CSR structure (indptr, column indices), and - with
dyadic coefficients and vectors, where every sum is exact in FP64 whatever its order - CSR
values and SpMV outputs.  Otherwise FP64 values agree within the summation bound
``(m + T) * eps * sum_j |H_ij| |x_j|`` (m entries in the row, T terms per element at most).
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import closed_forms as ocf
from oracle import lanczos as olz
from oracle import rowwise as orw
from oracle import subspace as osub

from _util import c2_keys, c3_parts, dyadic, dyadic_vector, heavy_hex_small, say

torch = pytest.importorskip("torch")
qsd = pytest.importorskip("paper_2603_18731_amd")

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qsd.lib()  # fail loudly if the library is missing


def _ham(keys, tl, **kw):
    sub = qsd.Subspace(keys, tl.n_qubits, **kw)
    op = qsd.operator_from_termlist(tl)
    return sub, op, qsd.SubspaceHamiltonian(sub, op)


def _to_np_keys(t):
    return t.cpu().numpy().view(np.uint64)


def _csr_gpu(H, index_type=qsd.INDEX_I64, dtype=None):
    ip, ix, dv = H.to_csr(index_type, dtype)
    torch.cuda.synchronize()
    return ip.cpu().numpy(), ix.cpu().numpy().astype(np.int64), dv.cpu().numpy()


# ------------------------------------------------------------------------ subspace / hash

@pytest.mark.parametrize("W,n,nkeys", [(1, 37, 5000 + 37), (1, 64, 3000), (2, 100, 7001), (4, 200, 4099),
                                       (8, 500, 1500), (16, 1024, 900)])
def test_subspace_keys_and_lookup(W, n, nkeys):
    say("subspace W=%d n=%d keys=%d" % (W, n, nkeys))
    rng = np.random.default_rng(W * 1000 + nkeys)
    vals = [int(v) for v in rng.integers(0, 2**62, size=nkeys)]
    vals = [(v * (1 + (v >> 7)) ** (W - 1)) & ((1 << n) - 1) for v in vals]
    vals += vals[: nkeys // 10]  # duplicates
    vals.append(0)
    keys = osub.ints_to_keys(vals, (n + 63) // 64)
    sub = qsd.Subspace(keys, n)
    expect = osub.canonical_keys(keys)
    got = _to_np_keys(sub.keys())
    assert sub.N == expect.shape[0]
    np.testing.assert_array_equal(got, expect)
    idx = sub.lookup(keys).cpu().numpy()
    canon = osub.keys_to_ints(expect)
    pos = {v: i for i, v in enumerate(canon)}
    np.testing.assert_array_equal(idx, [pos[v] for v in osub.keys_to_ints(keys)])
    # absent strings (including bits above n, which can never be members)
    absent = [(v ^ (1 << int(rng.integers(0, n)))) for v in vals[:500]]
    absent = [v for v in absent if v not in pos]
    ak = osub.ints_to_keys(absent, (n + 63) // 64)
    assert (sub.lookup(ak).cpu().numpy() == -1).all()
    mean, mx = sub.probe_stats()
    assert 1.0 <= mean < 3.0 and mx < 64


def test_subspace_errors():
    keys = np.array([[1], [1 << 40]], dtype=np.uint64)
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        qsd.Subspace(keys, 40)  # bit 40 set in a 40-qubit space
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        qsd.Subspace(np.zeros((0, 1), dtype=np.uint64), 10)
    sub = qsd.Subspace(np.array([[5]], dtype=np.uint64), 3)  # N = 1
    assert sub.N == 1 and sub.lookup(np.array([[5], [4]], dtype=np.uint64)).cpu().tolist() == [0, -1]


def test_subspace_sorted_input_flag():
    keys = np.arange(0, 3000, 3, dtype=np.uint64).reshape(-1, 1)
    sub = qsd.Subspace(keys, 12, assume_sorted_unique=True)
    np.testing.assert_array_equal(_to_np_keys(sub.keys()), keys)


# ------------------------------------------------------------------------------ cases

def _cases():
    """(name, term list, keys) at sizes the oracle finishes in seconds: several 256-row tiles
    and a ragged tail."""
    rng = np.random.default_rng(77)
    out = []
    c1 = wl.c1_tfim12()
    out.append(("tfim12", c1.ops, c1.keys))
    out.append(("xxz6x6_20k", wl.xxz_grid_6x6(), c2_keys(20_000)))
    out.append(("xxz6x6_pauli_5k", wl.xxz_terms(36, wl.grid_bonds(6, 6), 1.0, 0.8, ladder=False), c2_keys(5_003)))
    ops, keys = c3_parts(70, 70)
    out.append(("fermi16_70x70", ops, keys))
    hh_ops, hh_keys = heavy_hex_small(12_001)
    out.append(("heavyhex200_12k", hh_ops, hh_keys))
    # all seven letters, multi-word keys, random words (real elements: even #Y per word)
    n = 90
    terms = []
    for _ in range(60):
        m = int(rng.integers(1, 5))
        qs = rng.choice(n, size=m, replace=False)
        word = [(int(q), int(rng.choice([0, 1, 2, 3, 5, 6]))) for q in qs]
        terms.append((float(rng.normal()), word))
        terms.append((float(rng.normal()), [(int(q), 4) for q in rng.choice(n, size=2, replace=False)]))
    ref = int(rng.integers(0, 2**62))
    vals = {ref}
    while len(vals) < 3000:
        v = ref
        for q in rng.choice(n, size=int(rng.integers(1, 4)), replace=False):
            v ^= 1 << int(q)
        vals.add(v)
    out.append(("random7_n90", wl.TermList.from_terms(n, terms), osub.ints_to_keys(sorted(vals), 2)))
    return out


CASES = _cases()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_csr_exact_dyadic(case):
    name, tl, keys = case
    tl = dyadic(tl)
    say("csr dyadic", name, keys.shape)
    sub, op, H = _ham(keys, tl)
    ck = osub.canonical_keys(keys)
    ip_o, col_o, val_o = orw.rows_c(ck, tl)
    ip, ix, dv = _csr_gpu(H)
    np.testing.assert_array_equal(ip, ip_o)
    np.testing.assert_array_equal(ix, col_o)
    np.testing.assert_array_equal(dv, val_o.real)  # exact sums with dyadic coefficients
    ip32, ix32, _ = _csr_gpu(H, qsd.INDEX_I32)
    np.testing.assert_array_equal(ix32, col_o)
    d = H.diagonal().cpu().numpy()
    diag_o = np.array([val_o[a:b][col_o[a:b] == i][0].real for i, (a, b) in enumerate(zip(ip_o[:-1], ip_o[1:]))])
    np.testing.assert_array_equal(d, diag_o)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_matvec_exact_dyadic(case):
    name, tl, keys = case
    tl = dyadic(tl)
    say("matvec dyadic", name, keys.shape)
    sub, op, H = _ham(keys, tl)
    ck = osub.canonical_keys(keys)
    rng = np.random.default_rng(5)
    x = dyadic_vector(rng, sub.N)
    y_o = orw.matvec_c(ck, tl, x).real
    y = H.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    np.testing.assert_array_equal(y, y_o)
    # SpMM: 8 interleaved vectors, each equal to its own SpMV bit for bit
    X = dyadic_vector(rng, sub.N, nvec=8)
    Y_o = orw.matvec_c(ck, tl, X).real
    Y = H.matvec(torch.from_numpy(X).cuda()).cpu().numpy()
    np.testing.assert_array_equal(Y, Y_o)
    Y1 = np.stack([H.matvec(torch.from_numpy(np.ascontiguousarray(X[:, v])).cuda()).cpu().numpy() for v in range(8)], 1)
    np.testing.assert_array_equal(Y, Y1)
    # the widest SpMM kernels: 12 and 16 interleaved vectors
    for nv in (12, 16):
        X = dyadic_vector(rng, sub.N, nvec=nv)
        np.testing.assert_array_equal(H.matvec(torch.from_numpy(X).cuda()).cpu().numpy(), orw.matvec_c(ck, tl, X).real)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_matvec_fp64_bound(case):
    name, tl, keys = case
    say("matvec fp64", name, keys.shape)
    sub, op, H = _ham(keys, tl)
    ck = osub.canonical_keys(keys)
    rng = np.random.default_rng(6)
    x = rng.normal(size=sub.N)
    ip, cols, vals = orw.rows_c(ck, tl)
    y_o = orw.matvec_c(ck, tl, x).real
    y = H.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    tmax = max(1, int(np.diff(op.export()[4]).max()))
    absrow = np.add.reduceat(np.abs(vals) * np.abs(x[cols]), ip[:-1])
    m = np.diff(ip)
    bound = (m + tmax + 2) * EPS * (absrow + tmax * np.abs(tl.coef).max() * np.abs(x).max())
    assert (np.abs(y - y_o) <= bound).all(), float(np.max(np.abs(y - y_o) - bound))


@pytest.mark.parametrize("case", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_matvec_fp32(case):
    """FP32 elements and vectors, FP64 accumulation: with dyadic data narrow enough for FP32,
    the result is the exact value rounded once to FP32."""
    name, tl, keys = case
    tl = dyadic(tl, bits=8)
    say("matvec fp32", name, keys.shape)
    sub, op, H = _ham(keys, tl)
    ck = osub.canonical_keys(keys)
    rng = np.random.default_rng(7)
    X = dyadic_vector(rng, sub.N, bits=6, nvec=4)
    Y_o = orw.matvec_c(ck, tl, X).real.astype(np.float32)
    Y = H.matvec(torch.from_numpy(X.astype(np.float32)).cuda()).cpu().numpy()
    np.testing.assert_array_equal(Y, Y_o)
    ip, ix, dv = _csr_gpu(H, dtype=torch.float32)
    _, _, val_o = orw.rows_c(ck, tl)
    np.testing.assert_array_equal(dv, val_o.real.astype(np.float32))


def test_complex_operator():
    rng = np.random.default_rng(12)
    n = 10
    terms = []
    for _ in range(40):
        m = int(rng.integers(1, 4))
        qs = rng.choice(n, size=m, replace=False)
        word = [(int(q), int(rng.integers(0, 7))) for q in qs]
        c = complex(rng.normal(), rng.normal())
        terms.append((c, word))
        adj = [(q, {5: 6, 6: 5}.get(k, k)) for q, k in word]
        terms.append((c.conjugate(), adj))
    tl = dyadic(wl.TermList.from_terms(n, terms))
    keys = osub.ints_to_keys(sorted(rng.choice(1 << n, size=700, replace=False).tolist()), 1)
    say("complex n=10")
    sub, op, H = _ham(keys, tl)
    assert op.is_complex
    ck = osub.canonical_keys(keys)
    x = dyadic_vector(rng, sub.N, nvec=2) + 1j * dyadic_vector(rng, sub.N, nvec=2)
    Y_o = orw.matvec_c(ck, tl, x)
    Y = H.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    np.testing.assert_array_equal(Y, Y_o)
    ip_o, col_o, val_o = orw.rows_c(ck, tl)
    ip, ix, dv = _csr_gpu(H)
    np.testing.assert_array_equal(ip, ip_o)
    np.testing.assert_array_equal(ix, col_o)
    np.testing.assert_array_equal(dv, val_o)
    with pytest.raises(qsd.QsdError, match="DTYPE"):
        H.matvec(torch.zeros(sub.N, dtype=torch.float64, device="cuda"))


def test_hermitian_csr_c3():
    ops, keys = c3_parts(70, 70)
    tl = dyadic(ops)
    say("hermitian c3 70x70")
    sub, op, H = _ham(keys, tl)
    ip, ix, dv = _csr_gpu(H)
    import scipy.sparse as sp

    A = sp.csr_matrix((dv, ix, ip), shape=(sub.N, sub.N))
    D = (A - A.T).tocsr()
    assert abs(D).max() == 0
    S = (A != 0).astype(np.int8)
    assert (abs(S - S.T)).max() == 0


def test_ladder_ablation_same_matrix():
    """Without ladder-integer ranges every group is scanned term by term: same matrix."""
    ops, keys = c3_parts(40, 40)
    tl = dyadic(ops)
    say("ladder ablation")
    sub = qsd.Subspace(keys, tl.n_qubits)
    H1 = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(tl))
    H2 = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(tl, ladder_ints=False))
    a, b = _csr_gpu(H1), _csr_gpu(H2)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


# --------------------------------------------------------------------- full-size, sampled

def test_c2_full_sampled_rows():
    keys = c2_keys(1 << 20)
    tl = wl.xxz_grid_6x6()
    say("c2 full 2^20")
    sub, op, H = _ham(keys, tl)
    assert sub.N == 1 << 20
    ck = _to_np_keys(sub.keys())
    rng = np.random.default_rng(8)
    rows = np.sort(rng.choice(sub.N, size=20000, replace=False))
    rows[0], rows[-1] = 0, sub.N - 1
    # the oracle sorts the full key set itself
    ck_o = osub.canonical_keys(keys)
    np.testing.assert_array_equal(ck, ck_o)
    x = dyadic_vector(rng, sub.N)
    tld = dyadic(tl)
    Hd = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(tld))
    y_o = orw.matvec_c(ck_o, tld, x, rows).real
    # the default launch, then the one bench.py times (load 1/32, slot order, lockstep, filter
    # first, XCD remap: the autotuner's choice on this workload)
    y = Hd.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    np.testing.assert_array_equal(y[rows], y_o)
    sub.rehash(1 / 32)
    Hd.schedule = qsd.SCHED_ALL
    y15 = Hd.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    np.testing.assert_array_equal(y15, y)
    ip, ix, dv = _csr_gpu(Hd)
    ipo, co, vo = orw.rows_c(ck_o, tld, rows)
    for k, r in enumerate(rows[:3000]):
        np.testing.assert_array_equal(ix[ip[r]:ip[r + 1]], co[ipo[k]:ipo[k + 1]])
        np.testing.assert_array_equal(dv[ip[r]:ip[r + 1]], vo[ipo[k]:ipo[k + 1]].real)
    nnz = ip[-1]
    say("c2 nnz", nnz)
    assert nnz >= sub.N


def test_c3_full_sampled_rows():
    """The 2.25M-determinant fermionic workload, 400 sampled rows, without part filters, with
    them (split at the first beta qubit) through the product map and through the hash table,
    and in the launch bench.py times (the product map, filter-first schedule, XCD remap).  FP64 with 20-bit dyadic
    coefficients is exact; FP32 elements and vectors with 16-bit dyadic coefficients give the
    exact value rounded once (every element and every partial sum fits FP32 / FP64 exactly)."""
    ops, keys = c3_parts(1500, 1500)
    tl = dyadic(ops)
    tl16 = dyadic(ops, bits=16)
    say("c3 full 1500x1500")
    sub, op, H = _ham(keys, tl)
    H16 = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(tl16))
    assert sub.N == 2_250_000
    ck_o = osub.canonical_keys(keys)
    rng = np.random.default_rng(9)
    rows = np.sort(rng.choice(sub.N, size=400, replace=False))
    rows[0], rows[-1] = 0, sub.N - 1
    x = dyadic_vector(rng, sub.N)
    xd, x32 = torch.from_numpy(x).cuda(), torch.from_numpy(x.astype(np.float32)).cuda()
    y_o = orw.matvec_c(ck_o, tl, x, rows).real
    y16_o = orw.matvec_c(ck_o, tl16, x, rows).real.astype(np.float32)
    assert sub.hash_info()[2]  # an alpha x beta product: the map is found at build
    launches = [(0.125, 0, qsd.SCHED_FILTER_FIRST), (1 / 32, 16, qsd.SCHED_FILTER_FIRST),
                (1 / 32, 16, qsd.SCHED_FILTER_FIRST | qsd.SCHED_HASH_LOOKUP), (1 / 32, 16, qsd.SCHED_ALL),
                (0.125, 16, qsd.SCHED_FILTER_FIRST | qsd.SCHED_XCD_REMAP)]
    for load, split, sched in launches:
        say("c3 launch", load, split, sched)
        sub.rehash(load, split)
        H.schedule = H16.schedule = sched
        np.testing.assert_array_equal(H.matvec(xd).cpu().numpy()[rows], y_o)
        np.testing.assert_array_equal(H16.matvec(x32).cpu().numpy()[rows], y16_o)


def test_c3_full_csr_sampled_rows():
    """CSR of the full fermionic workload (1.74e9 entries, int32 columns): the two-pass build
    under part filters and the stored lower-triangle (mirrored) matrix, 300 sampled rows against
    the oracle's rows: structure exact, dyadic values exact."""
    ops, keys = c3_parts(1500, 1500)
    tl = dyadic(ops)
    say("c3 full CSR")
    sub, op, H = _ham(keys, tl)
    ck_o = osub.canonical_keys(keys)
    rng = np.random.default_rng(19)
    rows = np.sort(rng.choice(sub.N, size=300, replace=False))
    ipo, co, vo = orw.rows_c(ck_o, tl, rows)
    rows_t = torch.from_numpy(rows).cuda()

    def check(ip, ix, dv, label):
        a, b = ip[rows_t].cpu().numpy(), ip[rows_t + 1].cpu().numpy()
        for k in range(len(rows)):
            np.testing.assert_array_equal(ix[a[k]:b[k]].cpu().numpy().astype(np.int64), co[ipo[k]:ipo[k + 1]],
                                          err_msg=label)
            np.testing.assert_array_equal(dv[a[k]:b[k]].cpu().numpy(), vo[ipo[k]:ipo[k + 1]].real, err_msg=label)

    sub.rehash(1 / 32, 16)
    ip, ix, dv = H.to_csr(qsd.INDEX_I32)
    assert int(ip[-1]) == 1_738_419_792
    check(ip, ix, dv, "two-pass")
    del ip, ix, dv
    torch.cuda.empty_cache()
    A = qsd.CsrMatrix(H, qsd.INDEX_I32, lower_mirror=True)
    assert A.nnz == 1_738_419_792
    ip, ix, dv = A.export()
    del A
    check(ip, ix, dv, "lower-triangle")
    del ip, ix, dv
    torch.cuda.empty_cache()


def test_c4_full_sampled_rows():
    """The 5M-string 200-qubit heavy-hex workload (four key words), 5000 sampled rows: FP64
    8-vector SpMM and single vector, and FP32 (the coefficients 2 and 0.5 and 10-bit dyadic
    vectors are exact in FP32: the result is the exact value rounded once), in the default
    launch and in the launches the autotuner picks for it (load 1/32, slot order + lockstep +
    filter first, with and without the XCD remap)."""
    tl, keys = heavy_hex_small(5_000_000)
    say("c4 full 5M")
    tld = dyadic(tl)
    sub, op, H = _ham(keys, tld)
    assert sub.N == 5_000_000
    ck_o = osub.canonical_keys(keys)
    rng = np.random.default_rng(10)
    rows = np.sort(rng.choice(sub.N, size=5000, replace=False))
    X = dyadic_vector(rng, sub.N, nvec=8)
    Y_o = orw.matvec_c(ck_o, tld, X, rows).real
    Xd, X32 = torch.from_numpy(X).cuda(), torch.from_numpy(X.astype(np.float32)).cuda()
    x1, x132 = Xd[:, 0].contiguous(), X32[:, 0].contiguous()
    Y = H.matvec(Xd).cpu().numpy()
    np.testing.assert_array_equal(Y[rows], Y_o)
    for sched in (qsd.SCHED_ALL, qsd.SCHED_ALL & ~qsd.SCHED_XCD_REMAP):
        sub.rehash(1 / 32)
        H.schedule = sched
        np.testing.assert_array_equal(H.matvec(Xd).cpu().numpy(), Y)
        np.testing.assert_array_equal(H.matvec(x1).cpu().numpy()[rows], Y_o[:, 0])
        np.testing.assert_array_equal(H.matvec(X32).cpu().numpy()[rows], Y_o.astype(np.float32))
        np.testing.assert_array_equal(H.matvec(x132).cpu().numpy()[rows], Y_o[:, 0].astype(np.float32))


# ---------------------------------------------------------------------------- Lanczos

def test_lanczos_tfim12_closed_form():
    c1 = wl.c1_tfim12()
    sub, op, H = _ham(c1.keys, c1.ops)
    say("lanczos tfim12")
    e_exact = -2.0 / math.sin(math.pi / 24)
    side = torch.cuda.Stream()  # graph capture needs a non-default stream
    for use_graph in (False, True):
        with torch.cuda.stream(side):
            e, vec, info = H.lanczos(tol=1e-12, want_vector=True, use_graph=use_graph)
        torch.cuda.synchronize()
        assert abs(e - e_exact) / abs(e_exact) < 1e-10, (e, e_exact, info)
        assert info["explicit_residual"] < 1e-6
    e32, _, info32 = H.lanczos(tol=1e-7, spmv_dtype="f32", v0="random", seed=3)
    say("tfim12 fp32 rel err", abs(e32 - e_exact) / abs(e_exact))
    assert abs(e32 - e_exact) / abs(e_exact) < 1e-5


def test_lanczos_vs_oracle_c2_small():
    keys = c2_keys(20_000)
    tl = wl.xxz_grid_6x6()
    sub, op, H = _ham(keys, tl)
    ck = osub.canonical_keys(keys)
    A = orw.csr_c(ck, tl).real.tocsr()
    e_o, _, _ = olz.lanczos_ground(lambda v: A @ v, A.shape[0], tol=1e-13, max_iter=600)
    say("lanczos c2 20k oracle", e_o)
    e, _, info = H.lanczos(tol=1e-12, max_iter=600, v0="min_diag")
    assert abs(e - e_o) / abs(e_o) < 1e-10, (e, e_o, info)


def test_lanczos_xy_chain_closed_form():
    L, J, hz = 12, 1.0, 0.4
    tl = wl.xy_field_terms(L, [(i, i + 1) for i in range(L - 1)], J, hz)
    sub, op, H = _ham(wl.full_space(L), tl)
    e, _, info = H.lanczos(tol=1e-12, v0="random", seed=1)
    e_exact = ocf.xy_open_field_e0(L, J, hz)
    assert abs(e - e_exact) / abs(e_exact) < 1e-10


def test_lanczos_tiny_breakdown():
    keys = np.array([[0b0101], [0b1010], [0b0110]], dtype=np.uint64)
    tl = wl.xxz_terms(4, [(0, 1), (1, 2), (2, 3)], 1.0, 0.5)
    sub, op, H = _ham(keys, tl)
    e, _, info = H.lanczos(tol=1e-12)
    ck = osub.canonical_keys(keys)
    A = orw.csr_c(ck, tl).toarray().real
    assert abs(e - np.linalg.eigvalsh(A)[0]) < 1e-12
