"""Group trimming on the GPU: the smallest diagonal splitting equals the oracle's, and the
trimmed Hamiltonian's matrix equals the oracle's matrix of the oracle-trimmed term list (bit-exact
with dyadic coefficients); its ground energy moves by at most the removed groups' bounds."""
import numpy as np
import pytest

from oracle import lanczos as olz
from oracle import rowwise as orw
from oracle import subspace as osub
from oracle import trim as otr

from _util import c3_parts, dyadic, say

torch = pytest.importorskip("torch")
qsd = pytest.importorskip("paper_2603_18731_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qsd.lib()


def test_trimmed_fermionic_matrix():
    ops, keys = c3_parts(60, 60)
    tl = dyadic(ops)
    sub = qsd.Subspace(keys, tl.n_qubits)
    H = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(tl))
    ck = osub.canonical_keys(keys)
    A = orw.csr_c(ck, tl).tocsr()
    d = np.real(A.diagonal())
    lo, split = H.diag_splitting()
    assert lo == d.min() and split == otr.smallest_splitting(d)
    e_full, _, _ = H.lanczos(tol=1e-11, max_iter=600)
    B = otr.group_bounds(tl)
    for rel in (1e-4, 1e-3, 1e-2):
        Ht, thr = qsd.trimmed_hamiltonian(H, tl, rel)
        tlt = otr.trim_terms(tl, rel * split)
        ip, ix, dv = Ht.to_csr()
        ip_o, col_o, val_o = orw.rows_c(ck, tlt)
        np.testing.assert_array_equal(ip.cpu().numpy(), ip_o)
        np.testing.assert_array_equal(ix.cpu().numpy(), col_o)
        np.testing.assert_array_equal(dv.cpu().numpy(), np.real(val_o))
        e_t, _, _ = Ht.lanczos(tol=1e-11, max_iter=600)
        removed = sum(v for v in B.values() if v < thr)
        groups = Ht.op.n_groups
        say("trim rel %.0e: threshold %.3e, groups %d of %d, energy %.10f (full %.10f), removed bound %.3e" % (
            rel, thr, groups, H.op.n_groups, e_t, e_full, removed))
        assert abs(e_t - e_full) <= removed + 1e-9


def test_group_order_same_matrix():
    """Ordering groups by flip mask only (instead of weight, then mask) changes the evaluation
    order, not the matrix."""
    ops, keys = c3_parts(40, 40)
    tl = dyadic(ops)
    sub = qsd.Subspace(keys, tl.n_qubits)
    a = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(tl)).to_csr()
    b = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(tl, order_by_mask=True)).to_csr()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
