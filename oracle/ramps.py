"""RAMPS restricted to a sampled subspace (Supplement, Recursive algorithm for a minimal
perturbative subspace; Algorithm S1 with the S_full restriction of the same section).

Test infrastructure only: nothing in the library imports this module.

Given the Hamiltonian over the full sampled subspace S_full (here its matrix, rows and columns
in canonical order), an initial subspace S_0 (indices into S_full), a target energy E and a
tolerance tau, every state of S_0 starts a walk with prefactor 1/E.  A frontier entry (j, pre)
visits every off-diagonal matrix element H_jk of its row (the column of each off-diagonal group
that lies in S_full); the amplitude is

    amp = pre * |H_jk|^2 / (E - H_kk)

and when |amp| > tau the column joins the output and the next frontier with prefactor
amp / (E - H_kk).  Walks stop when a frontier is empty or after max_depth levels.  The output
is S_0 together with every column that was added.

Readings taken (the listing is silent or ambiguous on these):
* the next rows and their prefactors are parallel sequences: a column reached along several
  paths is carried once per path, each with its own prefactor (the output is a set);
* columns in S_0 are not followed (S_0 is the model space of the expansion, and with E equal to
  a diagonal element of S_0 the listing would divide by zero there);
* a zero denominator E - H_kk for a column outside S_0 follows IEEE arithmetic (the column is
  kept with an infinite amplitude; NaN amplitudes fail the test);
* the walks of different S_0 states are independent, so they may run as one frontier.
The arithmetic order is fixed: t = re*re + im*im; amp = (pre * t) / (E - H_kk);
next prefactor = amp / (E - H_kk).
"""
import numpy as np
import scipy.sparse as sp


def ramps_restricted(A, s0, E: float, tau: float, max_depth: int = 64):
    """Return ``(selected, levels)``: the sorted indices of S_out, and per level the list of
    ``(column, amplitude)`` pairs that passed the test (one per path)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    diag = np.real(A.diagonal()).astype(np.float64)
    s0 = sorted(set(int(i) for i in s0))
    in_s0 = np.zeros(n, dtype=bool)
    in_s0[s0] = True
    out = set(s0)
    frontier = [(i, np.float64(1.0) / np.float64(E)) for i in s0]
    levels = []
    depth = 0
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        while frontier and depth < max_depth:
            nxt = []
            passed = []
            for j, pre in frontier:
                a, b = A.indptr[j], A.indptr[j + 1]
                for k, h in zip(A.indices[a:b], A.data[a:b]):
                    k = int(k)
                    if k == j or in_s0[k]:
                        continue
                    re = np.float64(np.real(h))
                    im = np.float64(np.imag(h))
                    t = re * re + im * im
                    den = np.float64(E) - diag[k]
                    amp = (pre * t) / den
                    if abs(amp) > tau:
                        out.add(k)
                        nxt.append((k, amp / den))
                        passed.append((k, float(amp)))
            levels.append(passed)
            frontier = nxt
            depth += 1
    return sorted(out), levels
