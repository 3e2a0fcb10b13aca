"""RAMPS restricted to the sampled subspace (Supplement, Algorithm S1) on the GPU against the
oracle: the selected set, the number of levels and the number of paths are equal (dyadic
coefficients make every amplitude exact, so the tolerance tests take the same decisions); the
trimmed subspace holds exactly the selected strings and its ground energy is not below the full
subspace's (a subspace of S_full)."""
import numpy as np
import pytest

import workloads as wl
from oracle import ramps as ora
from oracle import rowwise as orw
from oracle import subspace as osub

from _util import c3_parts, dyadic, heavy_hex_small, say

torch = pytest.importorskip("torch")
qsd = pytest.importorskip("paper_2603_18731_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qsd.lib()


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
    if name == "fermi":
        ops, keys = c3_parts(60, 60)
        return keys, dyadic(ops)
    if name == "tfim12":
        c1 = wl.c1_tfim12()
        return c1.keys, dyadic(c1.ops)
    if name == "heavyhex":
        tl, keys = heavy_hex_small(20_000)
        return keys, dyadic(tl)
    return _complex_case()


# (case, start rule, E offset from the start's diagonal, taus, depths)
RUNS = [("fermi", "min", 0.0, (1e-5, 1e-7, 1e-9), (3, 8)),
        ("tfim12", "min2", 0.0, (1e-3, 1e-5), (2, 6)),
        ("heavyhex", "hub", -0.5, (1e-4, 1e-6), (6,)),
        ("complex", "min", -0.25, (1e-4, 1e-6), (5,))]


@pytest.mark.parametrize("name,rule,dE,taus,depths", RUNS)
def test_ramps_matches_oracle(name, rule, dE, taus, depths):
    keys, tl = _case(name)
    H = qsd.SubspaceHamiltonian(qsd.Subspace(keys, tl.n_qubits), qsd.operator_from_termlist(tl))
    A = orw.csr_c(osub.canonical_keys(keys), tl).tocsr()
    d = np.real(A.diagonal())
    if rule == "min":
        s0 = [int(np.argmin(d))]
    elif rule == "min2":
        s0 = [int(i) for i in np.argsort(d, kind="stable")[:2]]
    else:  # the row with the most off-diagonal entries
        s0 = [int(np.argmax(np.diff(A.indptr)))]
    E = float(d[s0[0]]) + dE
    for tau in taus:
        for depth in depths:
            sel, levels = ora.ramps_restricted(A, s0, E, tau, max_depth=depth)
            mask, info = H.ramps(s0, E, tau, max_depth=depth)
            got = np.nonzero(mask.cpu().numpy())[0].tolist()
            paths = sum(len(lv) for lv in levels)
            say(name, "tau", tau, "depth", depth, "selected", len(sel), "paths", paths, info)
            assert got == sel
            assert info["selected"] == len(sel)
            assert info["levels"] == len(levels)
            assert info["paths"] == paths
            assert info["truncated"] == int(len(levels) == depth and len(levels[-1]) > 0)


def test_ramps_trimmed_subspace():
    keys, tl = _case("fermi")
    sub = qsd.Subspace(keys, tl.n_qubits)
    op = qsd.operator_from_termlist(tl)
    H = qsd.SubspaceHamiltonian(sub, op)
    d = H.diagonal().cpu().numpy()
    s0 = [int(np.argmin(d))]
    mask, info = H.ramps(s0, float(d[s0[0]]), 1e-8, max_depth=10)
    small = sub.select(mask)
    assert small.N == info["selected"]
    ck = osub.canonical_keys(keys)
    np.testing.assert_array_equal(small.keys().cpu().numpy().view(np.uint64),
                                  ck[mask.cpu().numpy().astype(bool)])
    e_full, _, _ = H.lanczos(tol=1e-11, max_iter=600)
    Hs = qsd.SubspaceHamiltonian(small, op)
    e_small, _, _ = Hs.lanczos(tol=1e-11, max_iter=600)
    say("ramps trimmed", small.N, "of", sub.N, "energy", e_small, "full", e_full)
    assert e_small >= e_full - 1e-9 * abs(e_full)


def test_ramps_errors():
    keys, tl = _case("tfim12")
    H = qsd.SubspaceHamiltonian(qsd.Subspace(keys, tl.n_qubits), qsd.operator_from_termlist(tl))
    with pytest.raises(qsd.QsdError, match="CAPACITY"):
        H.ramps([0], -10.0, 0.0, max_depth=6, max_frontier=8)
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        H.ramps([H.N], -10.0, 1e-3)
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        H.ramps([0], -10.0, -1.0)
