"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here uses the GPU library.  Each test targets a specific way the oracle could be
wrong (orientation of the ladder letters, JW signs, a dropped term, the index order, the
row/column convention, the Lanczos recurrence).
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import alphabet as oal
from oracle import closed_forms as ocf
from oracle import dense as ode
from oracle import fermion as ofe
from oracle import lanczos as olz
from oracle import rowwise as orw
from oracle import subspace as osub

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LET = {"-": 5, "+": 6, "0": 1, "1": 2}


def _golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


# --------------------------------------------------------------------------- alphabet

def test_merge_rules_table_s1():
    """All 16 merge rules of Table S1 follow from the oracle's 2x2 letters."""
    rows = _golden_lines("merge_rules.txt")
    assert len(rows) == 16
    for a, b, res in rows:
        prod = oal.MATS[LET[a]] @ oal.MATS[LET[b]]
        if res == "null":
            assert np.count_nonzero(prod) == 0, (a, b)
        else:
            np.testing.assert_array_equal(prod, oal.MATS[LET[res]], err_msg=str((a, b)))


def test_pauli_algebra():
    Zm, Xm, Ym = oal.MATS[0], oal.MATS[3], oal.MATS[4]
    for m in (Zm, Xm, Ym):
        np.testing.assert_array_equal(m @ m, np.eye(2))
    np.testing.assert_array_equal(Xm @ Ym, 1j * Zm)
    np.testing.assert_array_equal(Ym @ Zm, 1j * Xm)
    # Z|0> = |0>: the computational basis state 0 has eigenvalue +1
    assert Zm[0, 0] == 1 and Zm[1, 1] == -1
    # projectors and ladders in terms of Paulis
    np.testing.assert_array_equal(oal.MATS[1], (np.eye(2) + Zm) / 2)
    np.testing.assert_array_equal(oal.MATS[2], (np.eye(2) - Zm) / 2)
    np.testing.assert_array_equal(oal.MATS[5], (Xm + 1j * Ym) / 2)
    np.testing.assert_array_equal(oal.MATS[6], (Xm - 1j * Ym) / 2)


# ---------------------------------------------------------------------------- fermions

def test_car_dense_n4():
    n = 4
    fs = ofe.dense_mode_ops(n)
    I = sp.identity(1 << n, format="csr")
    for i in range(n):
        for j in range(n):
            a = (fs[i] @ fs[j] + fs[j] @ fs[i]).toarray()
            assert np.count_nonzero(a) == 0
            b = (fs[i] @ fs[j].conj().T + fs[j].conj().T @ fs[i]).toarray()
            np.testing.assert_array_equal(b, (I.toarray() if i == j else 0 * b))


def test_jw_matches_pauli_formula():
    """f_j = 1/2 (X_j + i Y_j) Z_{j-1} ... Z_0, built from Pauli words on the dense route."""
    n = 4
    fs = ofe.dense_mode_ops(n)
    for j in range(n):
        zs = [(q, 0) for q in range(j)]
        m = 0.5 * ode.word_matrix(n, zs + [(j, 3)]) + 0.5j * ode.word_matrix(n, zs + [(j, 4)])
        np.testing.assert_array_equal(m.toarray(), fs[j].toarray())


def _random_fermion_terms(rng, n, nterms, maxlen=4):
    terms = []
    for _ in range(nterms):
        m = int(rng.integers(1, maxlen + 1))
        ops = [(int(rng.integers(0, n)), int(rng.integers(5, 7))) for _ in range(m)]
        terms.append((complex(rng.normal(), rng.normal()), ops))
    return terms


def test_direct_action_matches_dense():
    rng = np.random.default_rng(11)
    n = 5
    fs = ofe.dense_mode_ops(n)
    for c, ops in _random_fermion_terms(rng, n, 60):
        M = ofe.dense_term(n, ops, fs).toarray()
        for b in range(1 << n):
            r = ofe.row_action(b, ops)
            row = M[b]
            if r is None:
                assert np.count_nonzero(row) == 0
            else:
                s, col = r
                expect = np.zeros(1 << n)
                expect[col] = s
                np.testing.assert_array_equal(row, expect)


# ------------------------------------------------------------------ words and structure

def _random_qubit_terms(rng, n, nterms, maxlen=4, letters=range(7)):
    letters = list(letters)
    terms = []
    for _ in range(nterms):
        m = int(rng.integers(0, maxlen + 1))
        qs = rng.choice(n, size=m, replace=False)
        word = [(int(q), int(rng.choice(letters))) for q in sorted(qs)]
        terms.append((complex(rng.normal(), rng.normal()), word))
    return terms


def test_word_rows_nonzero_fraction():
    """A word with m projector/ladder letters is nonzero on exactly 2^(n-m) rows; a Pauli word
    has exactly one nonzero per row, at column row xor offmask (Methods, properties 1-2)."""
    rng = np.random.default_rng(5)
    n = 8
    for _ in range(40):
        [(c, word)] = _random_qubit_terms(rng, n, 1, maxlen=6)
        M = ode.word_matrix(n, word).toarray()
        m = sum(1 for _, k in word if k in (1, 2, 5, 6))
        nz_rows = np.count_nonzero(np.abs(M).sum(axis=1))
        assert nz_rows == 2 ** (n - m)
        assert all(np.count_nonzero(M[r]) <= 1 for r in range(1 << n))
        mask = sum(1 << q for q, k in word if k > 2)
        for r in range(1 << n):
            nzc = np.nonzero(M[r])[0]
            if nzc.size:
                assert nzc[0] == r ^ mask


def _dense_restrict_vs_rows(n, terms, values, fermionic):
    H = (ofe.dense_hamiltonian(n, terms) if fermionic else ode.qubit_hamiltonian(n, terms))
    Hs = ode.restrict(H, values)
    canon = osub.canonical(values)
    rows = orw.rows_python(canon, terms, fermionic)
    R = np.zeros_like(Hs)
    for i, r in enumerate(rows):
        for j, v in r:
            R[i, j] = v
        # every present entry is either nonzero or a cancellation; no nonzero is missing
        present = {j for j, _ in r}
        for j in np.nonzero(Hs[i])[0]:
            assert j in present
        assert i in present
    np.testing.assert_allclose(R, Hs, rtol=0, atol=1e-12)
    return rows


def test_rowwise_matches_dense_qubit():
    rng = np.random.default_rng(7)
    n = 7
    terms = _random_qubit_terms(rng, n, 40)
    values = rng.choice(1 << n, size=70, replace=False).tolist()
    _dense_restrict_vs_rows(n, terms, values, False)


def test_rowwise_matches_dense_fermion():
    rng = np.random.default_rng(8)
    n = 6
    terms = _random_fermion_terms(rng, n, 50)
    values = rng.choice(1 << n, size=40, replace=False).tolist()
    _dense_restrict_vs_rows(n, terms, values, True)


def test_structural_rule_cancellation():
    """XX + YY cancels on rows whose two bits agree; the entry stays present with 0.0."""
    terms = [(1.0, [(0, 3), (1, 3)]), (1.0, [(0, 4), (1, 4)])]
    rows = orw.rows_python([0, 1, 2, 3], terms, False)
    assert rows[0] == [(0, 0j), (3, 0j)]  # 00 -> 11 present, value 0
    assert rows[1] == [(1, 0j), (2, 2 + 0j)]


@pytest.mark.parametrize("fermionic", [False, True])
def test_c_matches_python(fermionic):
    rng = np.random.default_rng(21 + fermionic)
    for n, nvals in ((6, 30), (70, 300), (130, 200)):
        if fermionic:
            terms = _random_fermion_terms(rng, min(n, 70), 40)
        else:
            terms = _random_qubit_terms(rng, n, 40)
        # values: clustered around a reference so that columns land in the subspace
        ref = int(rng.integers(0, 1 << min(n, 62)))
        vals = {ref}
        while len(vals) < nvals:
            v = ref
            for q in rng.choice(n, size=int(rng.integers(1, 4)), replace=False):
                v ^= 1 << int(q)
            vals.add(v)
        canon = osub.canonical(vals)
        tl = wl.TermList.from_terms(n, terms, fermionic)
        keys = osub.ints_to_keys(canon, wl.n_words(n))
        indptr, cols, cv = orw.rows_c(keys, tl)
        rows = orw.rows_python(canon, terms, fermionic)
        for i, r in enumerate(rows):
            a, b = indptr[i], indptr[i + 1]
            assert cols[a:b].tolist() == [j for j, _ in r]
            np.testing.assert_allclose(cv[a:b], [v for _, v in r], rtol=1e-13, atol=1e-13)
        x = rng.normal(size=len(canon)) + 1j * rng.normal(size=len(canon))
        y = orw.matvec_c(keys, tl, x)
        yp = np.array([sum(v * x[j] for j, v in r) for r in rows])
        np.testing.assert_allclose(y, yp, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------------ index order

def test_canonical_index_bruteforce():
    rng = np.random.default_rng(3)
    for W in (1, 2, 3):
        vals = [int.from_bytes(rng.bytes(8 * W), "little") >> int(rng.integers(0, 40)) for _ in range(300)]
        vals += vals[:50]  # duplicates
        keys = osub.ints_to_keys(vals, W)
        ck = osub.canonical_keys(keys)
        assert osub.keys_to_ints(ck) == sorted(set(vals))


def test_msob_worked_example():
    for row_s, inds, tri in _golden_lines("msob_example.txt"):
        row = int(row_s, 2)
        mask = sum(1 << int(q) for q in inds.split(","))
        col = row ^ mask
        assert ("lower" if osub.is_lower(row, col) else "upper") == tri


# ----------------------------------------------------------------------- closed forms

def test_tfim12_closed_form_and_dense():
    e_formula = ocf.tfim_periodic_e0(12, 1.0, 1.0)
    assert abs(e_formula - (-2.0 / math.sin(math.pi / 24))) < 1e-12
    w = wl.c1_tfim12()
    H = ode.qubit_hamiltonian(12, list(w.ops.terms()))
    e = ode.ground_energy(ode.restrict(H, range(4096)).real)
    assert abs(e - e_formula) < 1e-11


@pytest.mark.parametrize("L,J,h,ladder", [(8, 1.0, 0.3, True), (9, 0.7, 1.1, False), (10, -0.5, 0.2, True)])
def test_xy_chain_closed_form(L, J, h, ladder):
    tl = wl.xy_field_terms(L, [(i, i + 1) for i in range(L - 1)], J, h, ladder=ladder)
    H = ode.qubit_hamiltonian(L, list(tl.terms()))
    e = ode.ground_energy(ode.restrict(H, range(1 << L)))
    assert abs(e - ocf.xy_open_field_e0(L, J, h)) < 1e-11


def test_quadratic_fermions_sector():
    rng = np.random.default_rng(4)
    n, N = 7, 3
    h = rng.normal(size=(n, n))
    h = (h + h.T) / 2
    terms = [(h[p, q], [(p, 6), (q, 5)]) for p in range(n) for q in range(n)]
    sector = [v for v in range(1 << n) if bin(v).count("1") == N]
    rows = orw.rows_python(sector, terms, True)
    M = np.zeros((len(sector), len(sector)), dtype=complex)
    for i, r in enumerate(rows):
        for j, v in r:
            M[i, j] = v
    assert abs(np.linalg.eigvalsh(M)[0] - ocf.quadratic_fermion_e0(h, N)) < 1e-12


def test_commuting_two_body_molecular_terms():
    """The generator's chemists'-notation expansion plus the oracle's direct action reproduce
    the closed-form spectrum of commuting one- and two-body parts (spinful, full sector)."""
    rng = np.random.default_rng(9)
    norb, na, nb = 4, 2, 1
    V, _ = np.linalg.qr(rng.normal(size=(norb, norb)))
    eps = rng.normal(size=norb)
    lam = rng.normal(size=norb)
    h = V @ np.diag(eps) @ V.T
    u = V @ np.diag(lam) @ V.T
    eri = np.einsum("pq,rs->pqrs", u, u)
    tl = wl.molecular_terms(h, eri)
    A = wl.weight_strings(norb, na)
    B = wl.weight_strings(norb, nb)
    keys = ((B[:, None] << np.uint64(norb)) | A[None, :]).reshape(-1, 1)
    ck = osub.canonical_keys(keys)
    Hs = orw.csr_c(ck, tl).toarray()
    np.testing.assert_allclose(Hs, Hs.conj().T, atol=1e-13)
    e = np.linalg.eigvalsh(Hs)[0]
    assert abs(e - ocf.commuting_two_body_e0_spin(eps, lam, na, nb)) < 1e-11


def test_commuting_two_body_spinless():
    """Spinless commuting parts: ``sum h_pq f+_p f_q + 1/2 sum (pq|rs) f+_p f+_r f_s f_q`` with
    ``h = V diag(eps) V^T`` and ``(pq|rs) = u_pq u_rs``, ``u = V diag(lam) V^T``, restricted to
    N particles by the oracle's direct action: its lowest eigenvalue is the closed form's minimum
    over occupations of the columns of V."""
    rng = np.random.default_rng(19)
    n, N = 6, 3
    V, _ = np.linalg.qr(rng.normal(size=(n, n)))
    eps = rng.normal(size=n)
    lam = rng.normal(size=n)
    h = V @ np.diag(eps) @ V.T
    u = V @ np.diag(lam) @ V.T
    terms = [(h[p, q], [(p, 6), (q, 5)]) for p in range(n) for q in range(n)]
    terms += [(0.5 * u[p, q] * u[r, s_], [(p, 6), (r, 6), (s_, 5), (q, 5)])
              for p in range(n) for q in range(n) for r in range(n) for s_ in range(n)]
    sector = [v for v in range(1 << n) if bin(v).count("1") == N]
    M = np.zeros((len(sector), len(sector)), dtype=complex)
    for i, row in enumerate(orw.rows_python(sector, terms, True)):
        for j, v in row:
            M[i, j] = v
    np.testing.assert_allclose(M, M.conj().T, atol=1e-12)
    e = np.linalg.eigvalsh(M)
    assert abs(e[0] - ocf.commuting_two_body_e0(eps, lam, N)) < 1e-11
    # every occupation is an eigenvalue: the closed form reproduces the whole spectrum
    from itertools import combinations

    spec = sorted(sum(eps[k] for k in occ) + sum(lam[a] * lam[b] for a, b in combinations(occ, 2))
                  for occ in combinations(range(n), N))
    np.testing.assert_allclose(e, spec, atol=1e-11)


# ---------------------------------------------------------------------------- Lanczos

def test_oracle_lanczos_tfim12():
    w = wl.c1_tfim12()
    ck = osub.canonical_keys(w.keys)
    H = orw.csr_c(ck, w.ops)
    assert abs(H - H.conj().T).max() == 0
    Hr = H.real.tocsr()
    e, x, it = olz.lanczos_ground(lambda v: Hr @ v, Hr.shape[0], tol=1e-13)
    e_exact = -2.0 / math.sin(math.pi / 24)
    assert abs(e - e_exact) / abs(e_exact) < 1e-12
    assert np.linalg.norm(Hr @ x - e * x) < 1e-6


def test_oracle_lanczos_xy_sector():
    L, J, hz = 10, 1.0, 0.4
    tl = wl.xy_field_terms(L, [(i, i + 1) for i in range(L - 1)], J, hz)
    ck = osub.canonical_keys(wl.full_space(L))
    H = orw.csr_c(ck, tl).real.tocsr()
    e, _, _ = olz.lanczos_ground(lambda v: H @ v, H.shape[0], v0=np.random.default_rng(0).normal(size=H.shape[0]),
                                 tol=1e-13)
    assert abs(e - ocf.xy_open_field_e0(L, J, hz)) < 1e-10


def test_workload_generators():
    n, edges = wl.heavy_hex_200()
    assert n == 200 and len(edges) == 229
    deg = np.bincount(np.array(edges).ravel(), minlength=n)
    assert deg.max() == 3
    col = wl.two_colouring(n, edges)
    assert int(col.sum()) == 117
    assert len(wl.grid_bonds(6, 6)) == 60
    k = wl.weight_sector_samples(36, 18, 5000, seed=2)
    assert len(set(k[:, 0].tolist())) == 5000
    assert all(bin(v).count("1") == 18 and v < (1 << 36) for v in k[:, 0].tolist())
    p = wl.product_subspace(16, 5, 5, 30, 20, seed=3)
    assert p.shape == (600, 1)
    h, eri = wl.molecular_integrals(6, seed=1)
    np.testing.assert_array_equal(h, h.T)
    for perm in ((1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)):
        np.testing.assert_array_equal(eri, eri.transpose(perm))


# ------------------------------------------------------------------ RAMPS (Supplement, Alg. S1)

def _chain4(h01):
    return np.array([[-5.0, h01, 0, 0], [np.conj(h01), -1.0, 0.2, 0], [0, 0.2, 0.5, 0.4], [0, 0, 0.4, 2.0]])


@pytest.mark.parametrize("h01", [0.3, 0.3j])
def test_ramps_chain_matches_eq_s1(h01):
    """On the tridiagonal 4-state chain with S_0 = {0} and E = H_00, the forward path's
    amplitudes at depths 1, 2, 3 are the three lines of the paper's recursive energy shift
    (Supplement, Eq. S1); |H_01|^2 (not H_01^2) enters, so a purely imaginary H_01 gives the
    same values."""
    from oracle import ramps as ora

    H = _chain4(h01)
    H00, H11, H22, H33 = H[0, 0].real, H[1, 1].real, H[2, 2].real, H[3, 3].real
    a01, a12, a23 = abs(H[0, 1]) ** 2, abs(H[1, 2]) ** 2, abs(H[2, 3]) ** 2
    line1 = a01 / (H00 * (H00 - H11))
    line2 = (1.0 / (H00 * (H00 - H11))) * (a01 / (H00 - H11)) * (a12 / (H00 - H22))
    line3 = (1.0 / (H00 * (H00 - H11) * (H00 - H22))) * (a01 / (H00 - H11)) * (a12 / (H00 - H22)) * (a23 / (H00 - H33))
    sel, levels = ora.ramps_restricted(sp.csr_matrix(H), [0], H00, 0.0, max_depth=3)
    assert sel == [0, 1, 2, 3]
    fwd = [dict(lv).get(k) for lv, k in zip(levels, (1, 2, 3))]
    np.testing.assert_allclose(fwd, [line1, line2, line3], rtol=1e-14)
    # back paths (2 -> 1) exist at depth 3; paths into S_0 are not followed
    assert all(k != 0 for lv in levels for k, _ in lv)


def _random_graph_h(n=60, seed=4):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=0.04, random_state=seed, data_rvs=lambda s: rng.normal(0, 0.3, s))
    M = sp.triu(M, 1)
    M = (M + M.T).tocsr()
    M.setdiag(np.sort(rng.normal(0, 3, n)) + 10.0)
    return M.tocsr()


def test_ramps_limits_and_ball():
    """tau = inf keeps S_0; tau = 0 keeps exactly the graph ball of radius max_depth around S_0
    (shortest paths, a library routine); the output shrinks as tau grows."""
    from scipy.sparse.csgraph import shortest_path

    from oracle import ramps as ora

    M = _random_graph_h()
    s0 = [3, 17]
    E = float(M[3, 3]) - 0.5
    sel, _ = ora.ramps_restricted(M, s0, E, np.inf, max_depth=10)
    assert sel == s0
    P = M.copy()
    P.setdiag(0)
    P.eliminate_zeros()
    dist = shortest_path((P != 0).astype(np.float64), unweighted=True, indices=s0).min(axis=0)
    for d in (1, 2, 3):
        sel, _ = ora.ramps_restricted(M, s0, E, 0.0, max_depth=d)
        assert sel == sorted(np.nonzero(dist <= d)[0].tolist()), d
    prev = None
    for tau in (1e-9, 1e-6, 1e-4, 1e-2):
        sel, _ = ora.ramps_restricted(M, s0, E, tau, max_depth=12)
        if prev is not None:
            assert set(sel) <= set(prev)
        prev = sel


# ------------------------------------------------------------------ group trimming

def test_trim_rules_qubit_and_fermion():
    from oracle import trim as otr

    tl = wl.TermList.from_terms(3, [(0.5, [(0, 3), (1, 3)]), (0.2, [(0, 4), (1, 4)]), (0.05, [(2, 3)]),
                                    (0.3, [(0, 0)]), (0.1, [(1, 1), (2, 6)])])
    B = otr.group_bounds(tl)
    assert B == {0b011: pytest.approx(0.7), 0b100: pytest.approx(0.05 + 0.1)}
    kept = otr.trim_terms(tl, 0.2)
    assert len(kept.coef) == 3  # XX, YY and the diagonal Z
    assert len(otr.trim_terms(tl, 0.0).coef) == 5
    assert len(otr.trim_terms(tl, 0.8).coef) == 1
    ft = wl.TermList.from_terms(4, [(0.4, [(0, 6), (1, 5)]), (0.4, [(1, 6), (0, 5)]), (1.0, [(0, 6), (0, 5)]),
                                    (0.01, [(2, 6), (3, 5)])], fermionic=True)
    Bf = otr.group_bounds(ft)
    assert Bf == {0b0011: pytest.approx(0.8), 0b1100: pytest.approx(0.01)}
    assert otr.smallest_splitting([3.0, 1.0, 1.0, 2.5]) == 1.5 and otr.smallest_splitting([2.0]) == 0.0


@pytest.mark.parametrize("fermionic", [False, True])
def test_trim_infinite_keeps_diagonal_and_weyl_bound(fermionic):
    """Trimming everything leaves exactly the diagonal of the dense matrix; any trimming moves
    the lowest eigenvalue by at most the norm of what was removed, which is at most the sum of
    the removed groups' bounds (Weyl's inequality)."""
    from oracle import trim as otr

    rng = np.random.default_rng(31 + fermionic)
    n = 6
    terms = []
    for _ in range(30):
        k = int(rng.integers(1, 4))
        qs = rng.choice(n, size=k, replace=not fermionic)
        codes = rng.integers(5, 7, size=k) if fermionic else rng.integers(0, 7, size=k)
        if not fermionic:
            qs = rng.choice(n, size=k, replace=False)
        word = [(int(q), int(c)) for q, c in zip(qs, codes)]
        c = float(rng.normal(0, 0.5))
        terms.append((c, word))
        terms.append((c, [(q, {5: 6, 6: 5}.get(cc, cc)) for q, cc in reversed(word)] if fermionic
                      else [(q, {5: 6, 6: 5}.get(cc, cc)) for q, cc in word]))
    tl = wl.TermList.from_terms(n, terms, fermionic=fermionic)

    def dense(t):
        if fermionic:
            return ofe.dense_hamiltonian(n, [(complex(t.coef[i]), list(zip(t.op_idx[t.term_ptr[i]:t.term_ptr[i + 1]].tolist(), t.op_code[t.term_ptr[i]:t.term_ptr[i + 1]].tolist()))) for i in range(len(t.coef))]).toarray()
        return ode.qubit_hamiltonian(n, [(complex(t.coef[i]), list(zip(t.op_idx[t.term_ptr[i]:t.term_ptr[i + 1]].tolist(), t.op_code[t.term_ptr[i]:t.term_ptr[i + 1]].tolist()))) for i in range(len(t.coef))]).toarray()

    Hf = dense(tl)
    H0 = dense(otr.trim_terms(tl, np.inf))
    np.testing.assert_allclose(H0, np.diag(np.diag(Hf)), atol=1e-12)
    B = otr.group_bounds(tl)
    for tol in sorted(B.values())[::5]:
        Ht = dense(otr.trim_terms(tl, tol))
        removed = sum(v for v in B.values() if v < tol)
        dE = abs(np.linalg.eigvalsh(Hf)[0] - np.linalg.eigvalsh(Ht)[0])
        nrm = np.linalg.norm(Hf - Ht, 2)
        assert dE <= nrm + 1e-12 and nrm <= removed + 1e-12
