"""The allocation-free batched SpMV (``qsd_matvec_batched_noalloc``) against the allocating one.

Both entry points plan the same request and tile tables and launch the same kernels; only where
the tables live differs (a fixed per-GPU device array instead of stream-ordered memory).  So
every output must equal ``qsd_matvec_batched``'s bitwise, on consecutive calls that reuse the
array (the second with a smaller input, whose tables only partly overwrite the first's), and
inputs beyond the array's stated limits must be rejected with CAPACITY.
"""
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


@pytest.fixture(scope="module")
def hams():
    c1 = wl.c1_tfim12()
    ops3, keys3 = c3_parts(40, 40)
    opsw, keysw = c3_parts(600, 4)
    hh, hex_keys = heavy_hex_small(4_000)
    return {
        "tfim12": _ham(c1.keys, c1.ops),
        "xxz20k": _ham(c2_keys(20_000), wl.xxz_grid_6x6()),
        "hex4k": _ham(hex_keys, hh),  # four key words: a launch of its own
        "fermi1600": _ham(keys3, ops3),
        "xxz3k": _ham(c2_keys(3_000), wl.xxz_grid_6x6()),
        "fermi2400": _ham(keysw, opsw),  # product tiles within its blocks of rows
    }


def _vectors(rng, hs, nvecs, dtype):
    xs = []
    for h, nv in zip(hs, nvecs):
        x = rng.standard_normal((h.N, nv)) if nv > 1 else rng.standard_normal(h.N)
        xs.append(torch.from_numpy(x).to(dtype).cuda())
    return xs


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_equals_batched_on_consecutive_calls(hams, dtype):
    rng = np.random.default_rng(21)
    calls = [
        (["tfim12", "xxz20k", "hex4k", "fermi1600", "xxz3k", "fermi2400"], [1, 3, 8, 16, 2, 1]),
        (["xxz3k", "tfim12"], [2, 1]),  # smaller: fewer requests, tiles and launches
    ]
    for names, nvecs in calls:
        hs = [hams[k] for k in names]
        xs = _vectors(rng, hs, nvecs, dtype)
        say("noalloc", dtype, names, nvecs)
        ref = qsd.matvec_batched(hs, xs)
        ys = [torch.full_like(x, float("nan")) for x in xs]
        qsd.matvec_batched_noalloc(hs, xs, ys)
        torch.cuda.synchronize()
        for name, y, r in zip(names, ys, ref):
            assert torch.equal(y, r), name


def test_noalloc_complex_chunks(hams):
    """Complex requests go in chunks of four vectors (one table entry per chunk)."""
    rng = np.random.default_rng(5)
    n = 10
    terms = []
    for _ in range(30):
        m = int(rng.integers(1, 4))
        qs = rng.choice(n, size=m, replace=False)
        word = [(int(q), int(rng.integers(0, 7))) for q in qs]
        c = complex(rng.normal(), rng.normal())
        terms.append((c, word))
        terms.append((c.conjugate(), [(q, {5: 6, 6: 5}.get(k, k)) for q, k in word]))
    tl = wl.TermList.from_terms(n, terms)
    from oracle import subspace as osub  # seeded key list only

    keys = osub.ints_to_keys(sorted(rng.choice(1 << n, size=700, replace=False).tolist()), 1)
    H = _ham(keys, tl)
    assert H.is_complex
    for nv in (9, 3):
        x = torch.from_numpy(rng.standard_normal((H.N, nv)) + 1j * rng.standard_normal((H.N, nv))).cuda()
        say("noalloc complex", nv)
        ref = qsd.matvec_batched([H], [x])[0]
        y = torch.full_like(x, complex("nan"))
        qsd.matvec_batched_noalloc([H], [x], [y])
        torch.cuda.synchronize()
        assert torch.equal(y, ref)


def test_noalloc_limits(hams):
    h = hams["tfim12"]
    x = torch.zeros(h.N, dtype=torch.float64, device="cuda")
    n = qsd.NOALLOC_MAX_REQUESTS + 1
    with pytest.raises(qsd.QsdError, match="CAPACITY"):
        qsd.matvec_batched_noalloc([h] * n, [x] * n, [torch.empty_like(x) for _ in range(n)])
    # row tiles: 17 requests of 2^20 rows are 69632 tiles of 256 rows
    big = _ham(c2_keys(1_048_576), wl.xxz_grid_6x6())
    assert 17 * ((big.N + 255) // 256) > qsd.NOALLOC_MAX_TILES
    xb = torch.zeros(big.N, dtype=torch.float64, device="cuda")
    with pytest.raises(qsd.QsdError, match="CAPACITY"):
        qsd.matvec_batched_noalloc([big] * 17, [xb] * 17, [xb.clone() for _ in range(17)])
    # within both limits the same call works and matches the allocating entry
    yb = [torch.empty_like(xb) for _ in range(16)]
    xs = [torch.from_numpy(np.random.default_rng(i).standard_normal(big.N)).cuda() for i in range(16)]
    qsd.matvec_batched_noalloc([big] * 16, xs, yb)
    ref = qsd.matvec_batched([big] * 16, xs)
    torch.cuda.synchronize()
    for a, b in zip(yb, ref):
        assert torch.equal(a, b)
