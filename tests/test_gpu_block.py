"""Block Lanczos (b = 4, 8) through the C-ABI: ground energies against closed forms and the
oracle within 1e-10 relative (FP64 SpMM) or 1e-5 (FP32 SpMM), bitwise reproducibility, the
invariant-subspace exit, and argument errors."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import closed_forms as ocf
from oracle import lanczos as olz
from oracle import rowwise as orw
from oracle import subspace as osub

from _util import c2_keys, heavy_hex_small, say

torch = pytest.importorskip("torch")
qsd = pytest.importorskip("paper_2603_18731_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qsd.lib()


def _ham(keys, tl):
    sub = qsd.Subspace(keys, tl.n_qubits)
    op = qsd.operator_from_termlist(tl)
    return qsd.SubspaceHamiltonian(sub, op)


def _oracle_e0(keys, tl):
    A = orw.csr_c(osub.canonical_keys(keys), tl).real.tocsr()
    e, _, _ = olz.lanczos_ground(lambda v: A @ v, A.shape[0], tol=1e-13, max_iter=800)
    return e


@pytest.mark.parametrize("block", [4, 8, 16])
def test_block_tfim12_closed_form(block):
    c1 = wl.c1_tfim12()
    H = _ham(c1.keys, c1.ops)
    e_exact = -2.0 / math.sin(math.pi / 24)
    side = torch.cuda.Stream()  # graph capture needs a non-default stream
    for use_graph in (False, True):
        with torch.cuda.stream(side):
            e, vec, info = H.lanczos(max_iter=60 if block < 16 else 40, tol=1e-11, block=block, want_vector=True,
                                     use_graph=use_graph, check_every=2)
        torch.cuda.synchronize()
        say("block", block, "graph", use_graph, e, info)
        assert info["converged"]
        assert abs(e - e_exact) / abs(e_exact) < 1e-10
        assert info["explicit_residual"] < 1e-5


@pytest.mark.parametrize("block", [8, 16])
def test_block_vs_oracle_xxz(block):
    """FP64 within 1e-10 of the oracle's energy, FP32 SpMM within 1e-5."""
    keys = c2_keys(20_000)
    tl = wl.xxz_grid_6x6()
    H = _ham(keys, tl)
    e_o = _oracle_e0(keys, tl)
    steps = 80 if block == 8 else 40
    e, _, info = H.lanczos(max_iter=steps, tol=1e-11, block=block, v0="min_diag")
    e32, _, info32 = H.lanczos(max_iter=steps, tol=1e-7, block=block, spmv_dtype="f32", v0="min_diag")
    say("block", block, "xxz20k", e, e32, e_o, info["iterations"], info32["iterations"])
    assert abs(e - e_o) / abs(e_o) < 1e-10
    assert abs(e32 - e_o) / abs(e_o) < 1e-5


@pytest.mark.parametrize("block", [8, 16])
def test_block_heavy_hex_four_words(block):
    """200 qubits (four key words): single-vector and block Lanczos within 1e-10 of the oracle's
    energy in FP64, block with FP32 SpMM within 1e-5."""
    tl, keys = heavy_hex_small(20_000)
    H = _ham(keys, tl)
    e_o = _oracle_e0(keys, tl)
    steps = 80 if block == 8 else 40
    e1, _, i1 = H.lanczos(tol=1e-11, max_iter=600)
    eb, _, ib = H.lanczos(max_iter=steps, tol=1e-11, block=block)
    eb32, _, _ = H.lanczos(max_iter=steps, tol=1e-7, block=block, spmv_dtype="f32")
    say("heavy-hex 20k: oracle", e_o, "single", e1, i1["iterations"], "block", block, eb, ib["iterations"], eb32)
    assert abs(eb - e_o) / abs(e_o) < 1e-10
    assert abs(e1 - e_o) / abs(e_o) < 1e-10
    assert abs(eb32 - e_o) / abs(e_o) < 1e-5


def test_block_f32_spmm():
    keys = c2_keys(20_000)
    tl = wl.xxz_grid_6x6()
    H = _ham(keys, tl)
    e_o = _oracle_e0(keys, tl)
    e, _, info = H.lanczos(max_iter=80, tol=1e-7, block=8, spmv_dtype="f32", v0="min_diag")
    err = abs(e - e_o) / abs(e_o)
    say("block f32 xxz20k rel err", err, info)
    assert info["converged"] and err < 1e-5


def test_block_reproducible():
    keys = c2_keys(20_000)
    H = _ham(keys, wl.xxz_grid_6x6())
    r1 = H.lanczos(max_iter=12, tol=1e-14, block=8, raise_on_nonconv=False)
    r2 = H.lanczos(max_iter=12, tol=1e-14, block=8, raise_on_nonconv=False)
    assert r1[0] == r2[0] and r1[2]["ritz_residual"] == r2[2]["ritz_residual"]
    assert not r1[2]["converged"] and r1[2]["iterations"] == 12


def test_block_invariant_subspace():
    """H = Z_0 + 0.5 has two eigenvalues: the block Krylov space is invariant after two steps
    and T is exact."""
    tl = wl.TermList.from_terms(12, [(1.0, [(0, 0)]), (0.5, [])])
    H = _ham(wl.full_space(12), tl)
    for block in (4, 8, 16):
        e, _, info = H.lanczos(max_iter=24, tol=1e-12, block=block, check_every=1)
        say("invariant", block, e, info)
        assert info["converged"] and info["ritz_residual"] == 0.0 and info["iterations"] == 2
        assert abs(e + 0.5) < 1e-13


def test_block_errors():
    c1 = wl.c1_tfim12()
    H = _ham(c1.keys, c1.ops)
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        H.lanczos(block=3)
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        H.lanczos(block=8, max_iter=81)
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        H.lanczos(block=16, max_iter=41)
    tiny = _ham(wl.full_space(3), wl.tfim_chain(3, 1.0, 1.0, True))  # 8 strings < 2 blocks of 8
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        tiny.lanczos(block=8)
    cx = _ham(wl.full_space(3), wl.TermList.from_terms(3, [(1.0, [(0, 4)]), (0.5, [(1, 3)])]))
    with pytest.raises(qsd.QsdError, match="UNSUPPORTED"):
        cx.lanczos(block=4)
    with pytest.raises(qsd.QsdError, match="NOT_CONVERGED"):
        H.lanczos(block=8, max_iter=2, tol=1e-14)
