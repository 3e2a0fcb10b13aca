"""Host-side tests of the library (no GPU): exported symbols, and the operator compiler
(fermion ordering/merging, extended Jordan-Wigner, combining, grouping) against the oracle's
dense routes."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as wl
from oracle import dense as ode
from oracle import fermion as ofe

qsd = pytest.importorskip("paper_2603_18731_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _lib_or_skip():
    if not os.path.exists(qsd.LIB_PATH):
        pytest.skip("libqsd.so not built")
    return qsd.lib()


def test_header_symbols_exported():
    _lib_or_skip()
    hdr = open(os.path.join(ROOT, "include", "qsd.h")).read()
    declared = sorted(set(re.findall(r"\b(qsd_[a-z0-9_]+)\s*\(", hdr)))
    assert len(declared) >= 20
    lib = ctypes.CDLL(qsd.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert set(qsd.EXPORTED) <= set(declared)


def _export_terms(op):
    tp, oi, oc, coef, gp, gl = op.export()
    terms = []
    for t in range(len(coef)):
        word = list(zip(oi[tp[t]:tp[t + 1]].tolist(), oc[tp[t]:tp[t + 1]].tolist()))
        terms.append((coef[t], word))
    return terms, gp, gl


def _random_qubit_tl(rng, n, nterms):
    terms = []
    for _ in range(nterms):
        m = int(rng.integers(0, 5))
        qs = rng.choice(n, size=m, replace=False)
        word = [(int(q), int(rng.integers(0, 7))) for q in qs]  # unsorted on purpose
        terms.append((complex(rng.normal(), rng.normal()), word))
    # duplicates to exercise combining
    terms += [(complex(rng.normal()), w) for _, w in terms[:5]]
    return wl.TermList.from_terms(n, terms)


def _random_fermion_tl(rng, n, nterms):
    terms = []
    for _ in range(nterms):
        m = int(rng.integers(1, 5))
        ops = [(int(rng.integers(0, n)), int(rng.integers(5, 7))) for _ in range(m)]
        terms.append((complex(rng.normal(), rng.normal()), ops))
    return wl.TermList.from_terms(n, terms, fermionic=True)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_compile_qubit_matches_dense(seed):
    _lib_or_skip()
    rng = np.random.default_rng(seed)
    n = 6
    tl = _random_qubit_tl(rng, n, 40)
    op = qsd.QubitOperator.from_termlist(tl)
    terms, gp, gl = _export_terms(op)
    A = ode.qubit_hamiltonian(n, list(tl.terms())).toarray()
    B = ode.qubit_hamiltonian(n, terms).toarray()
    np.testing.assert_allclose(B, A, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_compile_fermion_matches_dense(seed):
    _lib_or_skip()
    rng = np.random.default_rng(100 + seed)
    n = 6
    tl = _random_fermion_tl(rng, n, 60)
    op = qsd.FermionicOperator.from_termlist(tl)
    terms, gp, gl = _export_terms(op)
    for _, w in terms:
        assert all(k in (0, 1, 2, 5, 6) for _, k in w)  # JW output alphabet {Z, 0, 1, -, +}
    A = ofe.dense_hamiltonian(n, list(tl.terms())).toarray()
    B = ode.qubit_hamiltonian(n, terms).toarray()
    np.testing.assert_allclose(B, A, atol=1e-12)


def test_merge_rules_through_compiler():
    """Single-mode products of two letters compile to the Table S1 result."""
    _lib_or_skip()
    code = {"-": 5, "+": 6}
    letter_of = {5: "-", 6: "+", 1: "0", 2: "1"}
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "merge_rules.txt")) if ln.strip() and ln[0] != "#"]
    for a, b, res in rows:
        if a not in code or b not in code:
            continue  # projector inputs are not fermionic letters
        tl = wl.TermList.from_terms(3, [(1.0, [(1, code[a]), (1, code[b])])], fermionic=True)
        op = qsd.FermionicOperator.from_termlist(tl)
        terms, _, _ = _export_terms(op)
        if res == "null":
            assert terms == []
        else:
            assert len(terms) == 1 and terms[0][1] == [(1, {"-": 5, "+": 6, "0": 1, "1": 2}[res])]
            assert terms[0][0] == 1.0
    # three-operator products reproduce the projector rows, e.g. (f f^+) f = '0-' -> '-'
    for seq, res in (((5, 6, 5), 5), ((6, 5, 6), 6), ((5, 6, 5, 6), 1), ((6, 5, 6, 5), 2)):
        tl = wl.TermList.from_terms(2, [(1.0, [(0, c) for c in seq])], fermionic=True)
        terms, _, _ = _export_terms(qsd.FermionicOperator.from_termlist(tl))
        assert terms == [(1.0, [(0, res)])], (seq, terms)


@pytest.mark.parametrize("order", ["weight", "parts"])
def test_grouping_invariants(order):
    """Every group holds the terms of one flip mask, ladder ranges ascend inside a group, and
    the groups follow the requested order: (weight, mask), or by parts (halves of the qubits
    flipped: low only, both, high only; groups flipping both by high half, weight, low half;
    the others by weight, high half, low half).  Both orders hold the same groups."""
    _lib_or_skip()
    rng = np.random.default_rng(3)
    n = 8
    tl = _random_fermion_tl(rng, n, 200)
    op = qsd.FermionicOperator.from_termlist(tl, order_by_parts=order == "parts")
    terms, gp, gl = _export_terms(op)
    assert gp[0] == 0 and gp[-1] == len(terms)

    def off(word):
        return sum(1 << q for q, k in word if k > 2)

    for t in range(gp[0], gp[1]):
        assert off(terms[t][1]) == 0
    keys = []
    for g in range(1, len(gp) - 1):
        masks = {off(terms[t][1]) for t in range(gp[g], gp[g + 1])}
        assert len(masks) == 1
        m = masks.pop()
        assert m != 0
        lo, hi = m & ((1 << (n // 2)) - 1), m >> (n // 2)
        cls = 1 if lo and hi else (2 if hi else 0)
        wt = bin(m).count("1")
        keys.append((wt, m) if order == "weight" else ((cls, hi, wt, lo) if cls == 1 else (cls, wt, hi, lo)))
        if gl[g]:
            qs = [q for q in range(64) if m >> q & 1]
            lints = []
            for t in range(gp[g], gp[g + 1]):
                w = dict(terms[t][1])
                lints.append(sum((1 << k) for k, q in enumerate(qs) if w[q] == 6))
            assert lints == sorted(lints)
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    # the other order: the same groups with the same terms
    other = qsd.FermionicOperator.from_termlist(tl, order_by_parts=order != "parts")
    t2, gp2, _ = _export_terms(other)

    def group_set(ts, g):
        return {frozenset((complex(ts[t][0]), tuple(ts[t][1])) for t in range(g[k], g[k + 1]))
                for k in range(len(g) - 1)}

    assert group_set(terms, gp) == group_set(t2, gp2)


def test_compile_errors():
    _lib_or_skip()
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        qsd.QubitOperator(3, [0, 2], [1, 1], [0, 3], [1.0])  # repeated qubit
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        qsd.QubitOperator(3, [0, 1], [3], [0], [1.0])  # index >= n
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        qsd.QubitOperator(3, [0, 1], [0], [9], [1.0])  # bad code
    with pytest.raises(qsd.QsdError, match="NOT_HERMITIAN"):
        qsd.QubitOperator(3, [0, 1], [0], [6], [1.0], check_hermitian=True)  # lone raising letter
    herm = wl.TermList.from_terms(3, [(0.5, [(0, 6), (2, 5)]), (0.5, [(0, 5), (2, 6)]), (1.0, [(0, 4), (1, 4)])])
    op = qsd.QubitOperator.from_termlist(herm, check_hermitian=True)
    assert not op.is_complex  # c * (-i)^{#Y}: the YY term's elements are real
    op = qsd.QubitOperator(3, [0, 1], [1], [4], [1.0], check_hermitian=True)
    assert op.is_complex  # a single Y has imaginary elements
    tl = wl.TermList.from_terms(3, [(1j, [(1, 3)]), (-1j, [(1, 3)])])
    op = qsd.QubitOperator.from_termlist(tl)
    assert op.n_terms == 1  # cancelled words are kept


def test_molecular_compile_sizes():
    _lib_or_skip()
    h, eri = wl.molecular_integrals(16, seed=3)
    tl = wl.molecular_terms(h, eri)
    op = qsd.FermionicOperator.from_termlist(tl, check_hermitian=True)
    tp, oi, oc, coef, gp, gl = op.export()
    diag_terms = int(gp[1] - gp[0])
    sizes = np.diff(gp[1:])
    # number-conserving one- and two-body terms: off-diagonal structure on 2 or 4 qubits, all
    # groups with ladder ranges
    assert op.n_groups - 1 == 240 + 18040
    assert diag_terms == 528
    assert op.n_terms == 94848
    assert gl[1:].all()
    assert not op.is_complex
    assert sizes.max() == 62


@pytest.mark.parametrize("which", ["fermi", "xxz", "random_qubit"])
def test_trimming_selects_the_oracle_groups(which):
    """Compiling with trim_tol drops exactly the groups the oracle drops: the compiled operator
    equals the compile of the oracle-trimmed term list, at several thresholds."""
    from oracle import trim as otr

    if which == "fermi":
        h, eri = wl.molecular_integrals(6, 7)
        tl = wl.molecular_terms(h, eri)
    elif which == "xxz":
        tl = wl.xxz_grid_6x6()
    else:
        rng = np.random.default_rng(9)
        terms = []
        for _ in range(60):
            k = int(rng.integers(1, 4))
            qs = rng.choice(8, size=k, replace=False)
            terms.append((complex(rng.normal(0, 0.3), rng.normal(0, 0.3) * (k % 2)),
                          [(int(q), int(c)) for q, c in zip(qs, rng.integers(0, 7, size=k))]))
        tl = wl.TermList.from_terms(8, terms)
    B = sorted(otr.group_bounds(tl).values())
    for tol in (0.0, B[len(B) // 4], B[len(B) // 2], B[-1] * 1.0001):
        a = qsd.operator_from_termlist(tl, trim_tol=tol).export()
        b = qsd.operator_from_termlist(otr.trim_terms(tl, tol)).export()
        assert len(a[0]) == len(b[0])
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        qsd.operator_from_termlist(tl, trim_tol=-1.0)


def test_host_core_under_sanitizers(tmp_path):
    """The host core (operator compiler, hash and part-filter word generators, error state)
    built with g++ -fsanitize=address,undefined and driven by ``tests/host_sanitize.cpp``:
    random qubit and fermionic operators of 1 to 1024 qubits, every argument check, export
    round trips.  Any sanitizer report fails the test.  No HIP call is made."""
    import shutil
    import subprocess

    gxx = shutil.which("g++")
    rocm_inc = "/opt/rocm/include"
    if gxx is None or not os.path.isdir(os.path.join(rocm_inc, "hip")):
        pytest.skip("g++ or the HIP headers are not available")
    csrc = os.path.join(ROOT, "paper_2603_18731_amd", "csrc")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I" + rocm_inc,
             "-I" + os.path.join(ROOT, "include"), "-I" + csrc]
    srcs = [os.path.join(csrc, "opcompile.cpp"), os.path.join(csrc, "api.cpp"),
            os.path.join(ROOT, "tests", "host_sanitize.cpp")]
    exe = str(tmp_path / "host_sanitize")
    r = subprocess.run([gxx] + flags + srcs + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
                                               "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.strip().endswith("host core clean")


def test_projector_tails_layout():
    """Inside every ladder range of the compiled molecular operator, the terms whose only letter
    beyond the flipped qubits (and Z signs) is one '1' projector come last, one per qubit, in
    increasing qubit order: the layout that lets a row visit only the tail terms of its set
    qubits.  The compiled operator is still the input operator (dense check on 4 orbitals)."""
    _lib_or_skip()
    for norb in (4, 8):
        h, eri = wl.molecular_integrals(norb, seed=3)
        tl = wl.molecular_terms(h, eri)
        op = qsd.FermionicOperator.from_termlist(tl)
        terms, gp, gl = _export_terms(op)
        tails = 0
        for g in range(1, len(gp) - 1):
            if not gl[g]:
                continue
            flip = sorted({q for t in range(gp[g], gp[g + 1]) for q, k in terms[t][1] if k in (5, 6)})

            def lint(t):
                w = dict(terms[t][1])
                return sum(1 << i for i, q in enumerate(flip) if w[q] == 6)

            def spectator(t):
                rest = [(q, k) for q, k in terms[t][1] if q not in flip and k != 0]
                return rest[0][0] if len(rest) == 1 and rest[0][1] == 2 else None

            t = gp[g]
            while t < gp[g + 1]:
                u = t
                while u < gp[g + 1] and lint(u) == lint(t):
                    u += 1
                qs = [spectator(v) for v in range(t, u)]
                first = next((i for i, q in enumerate(qs) if q is not None), len(qs))
                tail = qs[first:]
                assert None not in tail, (g, qs)
                assert tail == sorted(set(tail)), (g, qs)
                tails += len(tail)
                t = u
        assert tails > 0
        if norb == 4:
            A = ofe.dense_hamiltonian(2 * norb, list(tl.terms())).toarray()
            B = ode.qubit_hamiltonian(2 * norb, terms).toarray()
            np.testing.assert_allclose(B, A, atol=1e-12)
    # a qubit operator whose terms arrive with the spectators first and out of order, beside a
    # plain term with a high Z and a term wanting a qubit clear (which stays in front)
    ws = [[(5, 2), (1, 5), (0, 6)], [(1, 5), (0, 6), (6, 0)], [(3, 2), (0, 6), (1, 5)], [(0, 6), (1, 5), (2, 1)],
          [(2, 2), (1, 5), (0, 6), (4, 0)], [(0, 5), (1, 6), (5, 2)], [(0, 5), (1, 6)]]
    tl = wl.TermList.from_terms(8, [(0.5 + 0.125 * i, w) for i, w in enumerate(ws)])
    op = qsd.QubitOperator.from_termlist(tl)
    terms, gp, gl = _export_terms(op)
    assert len(gp) == 3 and gl[1]
    words = [sorted(w) for _, w in terms[gp[1]:gp[2]]]
    assert words[:2] in ([[(0, 6), (1, 5), (2, 1)], [(0, 6), (1, 5), (6, 0)]],
                         [[(0, 6), (1, 5), (6, 0)], [(0, 6), (1, 5), (2, 1)]])
    assert words[2:5] == [[(0, 6), (1, 5), (2, 2), (4, 0)], [(0, 6), (1, 5), (3, 2)], [(0, 6), (1, 5), (5, 2)]]
    assert words[5:] == [[(0, 5), (1, 6)], [(0, 5), (1, 6), (5, 2)]]
    A = ode.qubit_hamiltonian(8, list(tl.terms())).toarray()
    B = ode.qubit_hamiltonian(8, terms).toarray()
    np.testing.assert_allclose(B, A, atol=1e-12)
