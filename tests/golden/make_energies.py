"""Writes ``energies.json``: ground energies of the large workloads from the CPU oracle alone.

For each workload the oracle builds ``H_S`` term by term (``oracle/rowwise``, plain C with
binary search over the sorted keys; no grouping, ladder integers or hashing) and finds its lowest
eigenvalue twice: with the oracle's Lanczos (full reorthogonalization, classical Gram-Schmidt
applied twice, ``oracle/lanczos``) and with SciPy's ARPACK ``eigsh`` (implicitly restarted
Lanczos, the eigensolver the paper's Results use).  Both must agree; the GPU tests compare
their ground energies with the recorded oracle value.  The paper has no closed form for these
Hamiltonians, so the two independent CPU eigensolvers on the oracle's matrix are the reference.

Run from the repository root:  ``python tests/golden/make_energies.py``  (about ten minutes on
eight cores; the 5M-string heavy-hex matrix needs ~10 GB of RAM for the Lanczos basis).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import scipy.sparse.linalg as sla  # noqa: E402

import workloads as wl  # noqa: E402
from oracle import lanczos as olz  # noqa: E402
from oracle import rowwise as orw  # noqa: E402
from oracle import subspace as osub  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "energies.json")


def ground(w, lanczos_iter):
    t0 = time.time()
    ck = osub.canonical_keys(w.keys)
    A = orw.csr_c(ck, w.ops).real.tocsr()
    t_csr = time.time() - t0
    print("# %s: N=%d nnz=%d (oracle CSR %.0f s)" % (w.name, A.shape[0], A.nnz, t_csr), flush=True)
    t0 = time.time()
    ev = sla.eigsh(A, k=1, which="SA", tol=0, return_eigenvectors=False)
    e_arpack = float(ev[0])
    print("#   ARPACK %.15f (%.0f s)" % (e_arpack, time.time() - t0), flush=True)
    t0 = time.time()
    e_lz, _, it = olz.lanczos_ground(lambda v: A @ v, A.shape[0], tol=1e-13, max_iter=lanczos_iter)
    print("#   oracle Lanczos %.15f in %d iterations (%.0f s)" % (e_lz, it, time.time() - t0), flush=True)
    rel = abs(e_lz - e_arpack) / abs(e_arpack)
    assert rel < 1e-11, (e_lz, e_arpack)
    return {"energy": e_lz, "energy_arpack": e_arpack, "rel_diff": rel, "N": int(A.shape[0]), "nnz": int(A.nnz),
            "lanczos_iterations": int(it)}


def main():
    res = {"note": "ground energies of H_S from the CPU oracle's term-by-term CSR: the oracle's Lanczos "
                   "(full reorthogonalization) and SciPy ARPACK eigsh; written by tests/golden/make_energies.py"}
    res["xxz6x6_w18_1048576"] = ground(wl.c2_xxz6x6(), 400)
    res["fermi16_300x300"] = ground(wl.c3_molecular(300, 300), 400)
    res["heavyhex200_5000000"] = ground(wl.c4_heavy_hex(), 400)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
