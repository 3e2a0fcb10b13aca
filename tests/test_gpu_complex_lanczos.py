"""Lanczos for a complex Hermitian operator (elements with imaginary parts from Y letters and
complex coefficients): the lowest eigenvalue of the oracle's dense matrix within 1e-10, matrix-free
and on the stored complex CSR, FP64 and with complex-FP32 SpMV (1e-5), with graph replay; the Ritz
vector's explicit residual is small."""
import numpy as np
import pytest

import workloads as wl
from oracle import rowwise as orw
from oracle import subspace as osub

from _util import say

torch = pytest.importorskip("torch")
qsd = pytest.importorskip("paper_2603_18731_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qsd.lib()


def _hermitian_case(n=11, nkeys=1500, seed=21):
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(60):
        m = int(rng.integers(1, 4))
        qs = rng.choice(n, size=m, replace=False)
        word = [(int(q), int(rng.integers(0, 7))) for q in qs]
        c = complex(rng.normal(), rng.normal())
        terms.append((c, word))
        terms.append((c.conjugate(), [(q, {5: 6, 6: 5}.get(k, k)) for q, k in word]))
    tl = wl.TermList.from_terms(n, terms)
    keys = osub.ints_to_keys(sorted(rng.choice(1 << n, size=nkeys, replace=False).tolist()), 1)
    return keys, tl


def test_complex_lanczos_energy():
    keys, tl = _hermitian_case()
    sub = qsd.Subspace(keys, tl.n_qubits)
    H = qsd.SubspaceHamiltonian(sub, qsd.operator_from_termlist(tl, check_hermitian=True))
    assert H.is_complex
    A = orw.csr_c(osub.canonical_keys(keys), tl).toarray()
    assert np.abs(A - A.conj().T).max() < 1e-12
    e_o = float(np.linalg.eigvalsh(A)[0])
    e, vec, info = H.lanczos(tol=1e-11, max_iter=600, want_vector=True)
    say("complex lanczos", e, e_o, info)
    assert abs(e - e_o) / abs(e_o) < 1e-10
    assert vec.dtype == torch.complex128 and info["explicit_residual"] < 1e-6
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        eg, _, _ = H.lanczos(tol=1e-11, max_iter=600, use_graph=True, v0="random", seed=5)
    torch.cuda.synchronize()
    assert abs(eg - e_o) / abs(e_o) < 1e-10
    e32, _, _ = H.lanczos(tol=1e-7, max_iter=600, spmv_dtype="f32")
    assert abs(e32 - e_o) / abs(e_o) < 1e-5
    C = qsd.CsrMatrix(H, lower_mirror=True)
    ec, _, _ = C.lanczos(tol=1e-11, max_iter=600, v0="min_diag")
    assert abs(ec - e_o) / abs(e_o) < 1e-10
    C64 = qsd.CsrMatrix(H, dtype=torch.complex64)
    ec32, _, _ = C64.lanczos(tol=1e-7, max_iter=600)
    assert abs(ec32 - e_o) / abs(e_o) < 1e-5
