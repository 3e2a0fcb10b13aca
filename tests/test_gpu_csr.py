"""Stored CSR operator through the C-ABI: the two-pass build and the lower-triangle build with
mirrored fill (most significant off-diagonal bit test) against the oracle's rows, bit-exact
with dyadic coefficients; CSR SpMV against the oracle's SpMV (exact with dyadic vectors); and
Lanczos / block Lanczos on the stored matrix against the oracle energy within 1e-10."""
import numpy as np
import pytest

import workloads as wl
from oracle import lanczos as olz
from oracle import rowwise as orw
from oracle import subspace as osub

from _util import c2_keys, c3_parts, dyadic, dyadic_vector, heavy_hex_small, say

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


def _complex_case():
    rng = np.random.default_rng(12)
    n = 10
    terms = []
    for _ in range(40):
        m = int(rng.integers(1, 4))
        qs = rng.choice(n, size=m, replace=False)
        word = [(int(q), int(rng.integers(0, 7))) for q in qs]
        c = complex(rng.normal(), rng.normal())
        terms.append((c, word))
        terms.append((c.conjugate(), [(q, {5: 6, 6: 5}.get(k, k)) for q, k in word]))
    tl = dyadic(wl.TermList.from_terms(n, terms))
    keys = osub.ints_to_keys(sorted(rng.choice(1 << n, size=700, replace=False).tolist()), 1)
    return keys, tl


def _case(name):
    if name == "tfim12":
        c1 = wl.c1_tfim12()
        return c1.keys, dyadic(c1.ops)
    if name == "xxz":
        return c2_keys(20_000), dyadic(wl.xxz_grid_6x6())
    if name == "fermi":
        ops, keys = c3_parts(40, 40)
        return keys, dyadic(ops)
    if name == "fermi_mid":
        ops, keys = c3_parts(12, 12)
        return keys, dyadic(ops)
    if name == "fermi_150":  # mean row ~40: 16 lanes per row
        ops, keys = c3_parts(150, 150)
        return keys, dyadic(ops)
    if name == "fermi_300":  # mean row ~100: a wave per row
        ops, keys = c3_parts(300, 300)
        return keys, dyadic(ops)
    if name == "heavyhex":
        tl, keys = heavy_hex_small(4_000)
        return keys, dyadic(tl)
    return _complex_case()


CASES = ["tfim12", "xxz", "fermi", "fermi_mid", "fermi_150", "fermi_300", "heavyhex", "complex"]


@pytest.mark.parametrize("lower", [False, True])
@pytest.mark.parametrize("name", CASES)
def test_csr_build_exact(name, lower):
    keys, tl = _case(name)
    H = _ham(keys, tl)
    A = qsd.CsrMatrix(H, qsd.INDEX_I32, lower_mirror=lower)
    ip, ix, dv = A.export()
    torch.cuda.synchronize()
    ck = osub.canonical_keys(keys)
    ip_o, col_o, val_o = orw.rows_c(ck, tl)
    say(name, "lower" if lower else "two-pass", "N", A.N, "nnz", A.nnz, "mean row", A.nnz / A.N)
    np.testing.assert_array_equal(ip.cpu().numpy(), ip_o)
    np.testing.assert_array_equal(ix.cpu().numpy().astype(np.int64), col_o)
    vals = dv.cpu().numpy()
    np.testing.assert_array_equal(vals, val_o if H.is_complex else val_o.real)


@pytest.mark.parametrize("name", CASES)
def test_csr_matvec_exact(name):
    keys, tl = _case(name)
    H = _ham(keys, tl)
    A = qsd.CsrMatrix(H, qsd.INDEX_I64, lower_mirror=True)
    ck = osub.canonical_keys(keys)
    rng = np.random.default_rng(5)
    for nvec in (1, 3, 16):
        x = dyadic_vector(rng, H.N, nvec=nvec)
        if H.is_complex:
            x = x + 1j * dyadic_vector(rng, H.N, nvec=nvec)
        xo = x if nvec > 1 else x[:, None]
        y_o = orw.matvec_c(ck, tl, xo)
        y = A.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
        np.testing.assert_array_equal(y if nvec > 1 else y[:, None], y_o)
        if nvec == 3:
            np.testing.assert_array_equal(H.matvec(torch.from_numpy(x).cuda()).cpu().numpy(), y)


def test_csr_f32_matches_rounding():
    keys, tl = _case("fermi")
    H = _ham(keys, tl)
    A = qsd.CsrMatrix(H, dtype=torch.float32)
    ck = osub.canonical_keys(keys)
    _, _, val_o = orw.rows_c(ck, tl)
    _, _, dv = A.export()
    np.testing.assert_array_equal(dv.cpu().numpy(), val_o.real.astype(np.float32))
    x = dyadic_vector(np.random.default_rng(2), H.N, dtype=np.float32)
    y = A.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    y_mf = H.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    np.testing.assert_array_equal(y, y_mf)  # dyadic: both exact before the final rounding
    with pytest.raises(qsd.QsdError, match="DTYPE"):
        A.matvec(torch.zeros(H.N, dtype=torch.float64, device="cuda"))


def test_csr_lanczos_energies():
    keys = c2_keys(20_000)
    tl = wl.xxz_grid_6x6()
    H = _ham(keys, tl)
    Ao = orw.csr_c(osub.canonical_keys(keys), tl).real.tocsr()
    e_o, _, _ = olz.lanczos_ground(lambda v: Ao @ v, Ao.shape[0], tol=1e-13, max_iter=800)
    A = qsd.CsrMatrix(H, lower_mirror=True)
    e1, vec, i1 = A.lanczos(tol=1e-11, max_iter=600, v0="min_diag", want_vector=True)
    e8, _, i8 = A.lanczos(tol=1e-11, max_iter=80, block=8, v0="min_diag")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        eg, _, ig = A.lanczos(tol=1e-11, max_iter=600, v0="min_diag", use_graph=True)
    torch.cuda.synchronize()
    say("csr lanczos xxz20k", e_o, e1, i1["iterations"], e8, i8["iterations"], eg)
    for e in (e1, e8, eg):
        assert abs(e - e_o) / abs(e_o) < 1e-10
    assert i1["explicit_residual"] < 1e-6
    A32 = qsd.CsrMatrix(H, dtype=torch.float32)
    e32, _, _ = A32.lanczos(tol=1e-7, max_iter=600, v0="min_diag")
    assert abs(e32 - e_o) / abs(e_o) < 1e-5
    with pytest.raises(qsd.QsdError, match="DTYPE"):
        A32.lanczos(spmv_dtype="f64")


def test_csr_lanczos_fermi():
    ops, keys = c3_parts(60, 60)
    H = _ham(keys, ops)
    Ao = orw.csr_c(osub.canonical_keys(keys), ops).real.tocsr()
    e_o = float(np.linalg.eigvalsh(Ao.toarray())[0])
    A = qsd.CsrMatrix(H, lower_mirror=True)
    e, _, info = A.lanczos(tol=1e-11, max_iter=600)
    say("csr lanczos fermi 60x60", e, e_o, info)
    assert abs(e - e_o) / abs(e_o) < 1e-10


def test_csr_errors():
    keys, tl = _case("complex")
    H = _ham(keys, tl)
    with pytest.raises(qsd.QsdError, match="DTYPE"):
        qsd.CsrMatrix(H, dtype=torch.float64)
    A = qsd.CsrMatrix(H)
    with pytest.raises(qsd.QsdError, match="UNSUPPORTED"):
        A.lanczos(block=4)  # block Lanczos is real only


@pytest.mark.parametrize("n,wmax", [(13, 7), (14, 7)])
def test_csr_rows_longer_than_lds(n, wmax):
    """Rows of 5812 and 9908 entries (every X word of weight 1..7 on the full space of 13 or 14
    qubits: every row reaches every column of weight distance <= 7), longer than the 4096 columns a
    row sort holds in LDS: the two-pass and the lower-triangle builds sort them in chunks; sampled
    rows (first, last, ragged middle) equal the oracle's, structure and dyadic values exactly."""
    import itertools

    rng = np.random.default_rng(n)
    terms = []
    for w in range(1, wmax + 1):
        for qs in itertools.combinations(range(n), w):
            terms.append((float(rng.integers(-16, 17) or 1) / 16.0, [(q, 3) for q in qs]))
    tl = wl.TermList.from_terms(n, terms)
    keys = osub.ints_to_keys(list(range(1 << n)), 1)
    say("long rows", n, "qubits,", len(terms), "groups")
    H = _ham(keys, tl)
    ck = osub.canonical_keys(keys)
    rows = np.array([0, 1, 777, (1 << n) // 2, (1 << n) - 1])
    ipo, co, vo = orw.rows_c(ck, tl, rows)
    assert (np.diff(ipo) > 4096).all()
    rows_t = torch.from_numpy(rows).cuda()

    def check(ip, ix, dv, label):
        a, b = ip[rows_t].cpu().numpy(), ip[rows_t + 1].cpu().numpy()
        for k in range(len(rows)):
            np.testing.assert_array_equal(ix[a[k]:b[k]].cpu().numpy().astype(np.int64), co[ipo[k]:ipo[k + 1]],
                                          err_msg=label)
            np.testing.assert_array_equal(dv[a[k]:b[k]].cpu().numpy(), vo[ipo[k]:ipo[k + 1]].real, err_msg=label)

    ip, ix, dv = H.to_csr(qsd.INDEX_I32)
    check(ip, ix, dv, "two-pass")
    del ip, ix, dv
    A = qsd.CsrMatrix(H, qsd.INDEX_I64, lower_mirror=True)
    ip, ix, dv = A.export()
    check(ip, ix, dv, "lower-triangle")
    del A, ip, ix, dv
    torch.cuda.empty_cache()
