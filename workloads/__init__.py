"""Seeded synthetic inputs for the subspace-Hamiltonian SpMV.

This module only *writes down* inputs: bit-string subspaces and operator term lists in the
flat CSR-of-terms form that both the GPU library and the CPU oracle consume.  It holds none
of the method's arithmetic (no Jordan-Wigner transform, no merging, grouping, hashing or
matrix evaluation).

Conventions shared by every consumer:

* Qubit ``q`` of a bit-string is bit ``q % 64`` of 64-bit word ``q // 64`` (little-endian
  words; "bit indexing starts from the right", Supplemental Material, MSOB section).
  A subspace is a ``uint64`` array of shape ``[n][W]`` with ``W = ceil(n_qubits / 64)``.
* Operator letters use the extended-alphabet codes of the Methods section (Qubit
  Hamiltonians): ``Z=0, '0'=1, '1'=2, X=3, Y=4, '-'=5, '+'=6``.  For fermionic term lists
  code 5 is the annihilator ``f`` and code 6 the creator ``f^dagger``, listed in product
  order (leftmost operator first).
* A term list is ``term_ptr[T+1]`` (int64), ``op_idx[nops]`` (int32), ``op_code[nops]``
  (uint8) and ``coef[T]`` (complex128).  An empty word is the identity.

Random draws use ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import combinations
import math

import numpy as np

Z, P0, P1, X, Y, LOWER, RAISE = 0, 1, 2, 3, 4, 5, 6
F_ANN, F_CRE = LOWER, RAISE


@dataclass
class TermList:
    """Flat CSR-of-terms operator input."""

    n_qubits: int
    term_ptr: np.ndarray  # int64 [T+1]
    op_idx: np.ndarray  # int32 [nops]
    op_code: np.ndarray  # uint8 [nops]
    coef: np.ndarray  # complex128 [T]
    fermionic: bool = False

    @property
    def n_terms(self) -> int:
        return int(self.term_ptr.shape[0] - 1)

    def terms(self):
        """Iterate ``(coef, [(idx, code), ...])`` in input order."""
        for t in range(self.n_terms):
            a, b = int(self.term_ptr[t]), int(self.term_ptr[t + 1])
            yield complex(self.coef[t]), list(zip(self.op_idx[a:b].tolist(), self.op_code[a:b].tolist()))

    @staticmethod
    def from_terms(n_qubits: int, terms, fermionic: bool = False) -> "TermList":
        ptr = [0]
        idx: list[int] = []
        code: list[int] = []
        coef: list[complex] = []
        for c, word in terms:
            for q, k in word:
                idx.append(int(q))
                code.append(int(k))
            ptr.append(len(idx))
            coef.append(complex(c))
        return TermList(
            n_qubits,
            np.asarray(ptr, dtype=np.int64),
            np.asarray(idx, dtype=np.int32),
            np.asarray(code, dtype=np.uint8),
            np.asarray(coef, dtype=np.complex128),
            fermionic,
        )


def n_words(n_qubits: int) -> int:
    return max(1, (n_qubits + 63) // 64)


def ints_to_keys(values, n_qubits: int) -> np.ndarray:
    """Python ints -> ``uint64[n][W]`` little-endian words."""
    W = n_words(n_qubits)
    out = np.zeros((len(values), W), dtype=np.uint64)
    for i, v in enumerate(values):
        v = int(v)
        for w in range(W):
            out[i, w] = (v >> (64 * w)) & 0xFFFFFFFFFFFFFFFF
    return out


def keys_to_ints(keys: np.ndarray) -> list[int]:
    keys = np.asarray(keys, dtype=np.uint64)
    if keys.ndim == 1:
        keys = keys[:, None]
    out = []
    for row in keys:
        v = 0
        for w in range(keys.shape[1] - 1, -1, -1):
            v = (v << 64) | int(row[w])
        out.append(v)
    return out


# --------------------------------------------------------------------------- operators

def tfim_chain(L: int = 12, J: float = 1.0, h: float = 1.0, periodic: bool = True) -> TermList:
    """Transverse-field Ising chain ``H = -J sum Z_i Z_{i+1} - h sum X_i``."""
    terms = []
    nb = L if periodic else L - 1
    for i in range(nb):
        j = (i + 1) % L
        a, b = min(i, j), max(i, j)
        terms.append((-J, [(a, Z), (b, Z)]))
    for i in range(L):
        terms.append((-h, [(i, X)]))
    return TermList.from_terms(L, terms)


def grid_bonds(rows: int, cols: int) -> list[tuple[int, int]]:
    """Open ``rows x cols`` grid, site ``cols*r + c``; horizontal then vertical bonds."""
    bonds = []
    for r in range(rows):
        for c in range(cols - 1):
            bonds.append((cols * r + c, cols * r + c + 1))
    for r in range(rows - 1):
        for c in range(cols):
            bonds.append((cols * r + c, cols * (r + 1) + c))
    return bonds


def xxz_terms(n: int, bonds, jxy: float, jz: float, ladder: bool = True) -> TermList:
    """``sum_<ij> jxy (X_i X_j + Y_i Y_j) + jz Z_i Z_j``.

    With ``ladder=True`` the flip-flop part is written as ``2 jxy (+_i -_j + -_i +_j)``,
    otherwise with Pauli X and Y letters.
    """
    terms = []
    for i, j in bonds:
        a, b = min(i, j), max(i, j)
        if ladder:
            terms.append((2.0 * jxy, [(a, RAISE), (b, LOWER)]))
            terms.append((2.0 * jxy, [(a, LOWER), (b, RAISE)]))
        else:
            terms.append((jxy, [(a, X), (b, X)]))
            terms.append((jxy, [(a, Y), (b, Y)]))
        if jz != 0.0:
            terms.append((jz, [(a, Z), (b, Z)]))
    return TermList.from_terms(n, terms)


def xy_field_terms(n: int, edges, J: float, hz: float, ladder: bool = True) -> TermList:
    """``sum_E J (X_i X_j + Y_i Y_j) + hz sum_i Z_i``."""
    base = xxz_terms(n, edges, J, 0.0, ladder=ladder)
    terms = list(base.terms())
    for i in range(n):
        if hz != 0.0:
            terms.append((hz, [(i, Z)]))
    return TermList.from_terms(n, terms)


def xxz_grid_6x6() -> TermList:
    """2D XXZ on the open 6x6 grid, ``Jxy = 1``, ``Jz = 0.8``, ladder form."""
    return xxz_terms(36, grid_bonds(6, 6), 1.0, 0.8, ladder=True)


def heavy_hex_200():
    """Heavy-hex-style graph on 200 qubits.

    Six chains of 28 qubits; bridge qubits join chain r and r+1 at columns ``c = 0 mod 4``
    (even r) or ``c = 2 mod 4`` (odd r), 7 per gap.  Numbering is row-major with chain r's
    qubits followed by gap r's bridges (203 sites); sites >= 200 are dropped.
    Returns ``(n, edges)``.
    """
    rows, chain, keep = 6, 28, 200
    site = {}
    nxt = 0
    for r in range(rows):
        for c in range(chain):
            site[("q", r, c)] = nxt
            nxt += 1
        if r < rows - 1:
            cs = range(0, chain, 4) if r % 2 == 0 else range(2, chain, 4)
            for c in cs:
                site[("b", r, c)] = nxt
                nxt += 1
    edges = []
    for r in range(rows):
        for c in range(chain - 1):
            edges.append((site[("q", r, c)], site[("q", r, c + 1)]))
    for (kind, r, c), s in site.items():
        if kind == "b":
            edges.append((site[("q", r, c)], s))
            edges.append((s, site[("q", r + 1, c)]))
    edges = [(min(a, b), max(a, b)) for a, b in edges if a < keep and b < keep]
    return keep, sorted(edges)


def two_colouring(n: int, edges) -> np.ndarray:
    """BFS 2-colouring from site 0 (colour of every site; raises if not bipartite)."""
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    col = -np.ones(n, dtype=np.int64)
    for s in range(n):
        if col[s] >= 0:
            continue
        col[s] = 0
        stack = [s]
        while stack:
            u = stack.pop()
            for v in adj[u]:
                if col[v] < 0:
                    col[v] = 1 - col[u]
                    stack.append(v)
                elif col[v] == col[u]:
                    raise ValueError("graph is not bipartite")
    return col


def heavy_hex_xy_field() -> TermList:
    n, edges = heavy_hex_200()
    return xy_field_terms(n, edges, 1.0, 0.5, ladder=True)


# ----------------------------------------------------------------- molecular (fermionic)

def molecular_integrals(norb: int = 16, seed: int = 3, h_scale: float = 0.1, g_scale: float = 0.01):
    """Random real integrals: ``h`` symmetric ~ N(0, h_scale); ``(pq|rs)`` with the 8-fold
    permutational symmetry, one normal draw (std ``g_scale``) per symmetry orbit."""
    rng = np.random.default_rng(seed)
    h = rng.normal(0.0, h_scale, size=(norb, norb))
    h = np.triu(h) + np.triu(h, 1).T
    npair = norb * (norb + 1) // 2
    pair_vals = rng.normal(0.0, g_scale, size=(npair, npair))
    pair_vals = np.triu(pair_vals) + np.triu(pair_vals, 1).T
    pid = np.zeros((norb, norb), dtype=np.int64)
    k = 0
    for p in range(norb):
        for q in range(p, norb):
            pid[p, q] = pid[q, p] = k
            k += 1
    eri = pair_vals[pid[:, :, None, None], pid[None, None, :, :]]
    return h, eri


def molecular_terms(h: np.ndarray, eri: np.ndarray, h0: float = 0.0) -> TermList:
    """Second-quantized molecular Hamiltonian (chemists' notation) as a fermionic term list.

    ``H = h0 + sum_{pq,s} h_pq f+_{ps} f_{qs}
          + 1/2 sum_{pqrs,s,t} (pq|rs) f+_{ps} f+_{rt} f_{st} f_{qs}``
    Spin orbital ``(p, alpha)`` is mode ``p``; ``(p, beta)`` is mode ``p + norb``.
    Every index combination is listed (products that vanish are kept; the compiler drops
    them).
    """
    norb = h.shape[0]
    n = 2 * norb
    terms = []
    if h0 != 0.0:
        terms.append((h0, []))
    for s in range(2):
        off = s * norb
        for p in range(norb):
            for q in range(norb):
                c = float(h[p, q])
                if c != 0.0:
                    terms.append((c, [(p + off, F_CRE), (q + off, F_ANN)]))
    for s in range(2):
        for t in range(2):
            os_, ot = s * norb, t * norb
            for p in range(norb):
                for q in range(norb):
                    for r in range(norb):
                        for u in range(norb):
                            c = 0.5 * float(eri[p, q, r, u])
                            if c != 0.0:
                                terms.append((c, [(p + os_, F_CRE), (r + ot, F_CRE),
                                                  (u + ot, F_ANN), (q + os_, F_ANN)]))
    return TermList.from_terms(n, terms, fermionic=True)


def weight_strings(nbits: int, weight: int) -> np.ndarray:
    """All ``nbits``-bit strings of the given Hamming weight, ascending (uint64)."""
    vals = []
    for comb in combinations(range(nbits), weight):
        v = 0
        for b in comb:
            v |= 1 << b
        vals.append(v)
    return np.asarray(sorted(vals), dtype=np.uint64)


def product_subspace(norb: int = 16, nalpha: int = 5, nbeta: int = 5, na: int = 1500,
                     nb: int = 1500, seed: int = 3) -> np.ndarray:
    """alpha x beta Cartesian-product determinants; key = ``beta << norb | alpha``.

    ``na`` alpha and ``nb`` beta strings are drawn without replacement from the strings of
    the right weight (same ``seed`` stream as the integrals follow separately)."""
    assert 2 * norb <= 64
    rng = np.random.default_rng(seed + 1000)
    A = weight_strings(norb, nalpha)
    B = weight_strings(norb, nbeta)
    a = A[rng.choice(A.shape[0], size=min(na, A.shape[0]), replace=False)]
    b = B[rng.choice(B.shape[0], size=min(nb, B.shape[0]), replace=False)]
    keys = (b[:, None] << np.uint64(norb)) | a[None, :]
    return keys.reshape(-1, 1).astype(np.uint64)


# ------------------------------------------------------------------------- subspaces

def full_space(n_qubits: int) -> np.ndarray:
    assert n_qubits <= 24
    return np.arange(1 << n_qubits, dtype=np.uint64).reshape(-1, 1)


def weight_sector_samples(nbits: int = 36, weight: int = 18, count: int = 1 << 20,
                          seed: int = 2, batch: int = 1 << 19) -> np.ndarray:
    """``count`` distinct strings drawn uniformly from the weight sector, kept in draw order.

    Each draw picks the ``weight`` smallest of ``nbits`` uniform variates (a uniform random
    subset); duplicates are rejected.
    """
    assert nbits <= 64
    rng = np.random.default_rng(seed)
    seen: dict[int, None] = {}
    pows = (np.uint64(1) << np.arange(nbits, dtype=np.uint64))
    while len(seen) < count:
        u = rng.random((batch, nbits))
        sel = np.argpartition(u, weight - 1, axis=1)[:, :weight]
        vals = np.bitwise_or.reduce(pows[sel], axis=1)
        for v in vals.tolist():
            if v not in seen:
                seen[v] = None
                if len(seen) == count:
                    break
    return np.fromiter(seen.keys(), dtype=np.uint64, count=count).reshape(-1, 1)


def reference_flip_samples(n_qubits: int, ref_bits: np.ndarray, count: int, seed: int = 4,
                           kmax: int = 6, batch: int = 1 << 20) -> np.ndarray:
    """``count`` distinct strings ``ref XOR (k distinct uniform flips)``, ``k ~ U{1..kmax}``,
    kept in draw order.  ``ref_bits`` is a 0/1 array of length ``n_qubits``."""
    W = n_words(n_qubits)
    ref = np.zeros(W, dtype=np.uint64)
    for q in np.nonzero(ref_bits)[0]:
        ref[q // 64] |= np.uint64(1) << np.uint64(q % 64)
    rng = np.random.default_rng(seed)
    out = []
    seen: set = set()
    total = 0
    while total < count:
        k = rng.integers(1, kmax + 1, size=batch)
        pos = rng.integers(0, n_qubits, size=(batch, kmax))
        active = np.arange(kmax)[None, :] < k[:, None]
        while True:
            bad = np.zeros(batch, dtype=bool)
            for i in range(kmax):
                for j in range(i + 1, kmax):
                    bad |= active[:, j] & (pos[:, i] == pos[:, j])
            if not bad.any():
                break
            pos[bad] = rng.integers(0, n_qubits, size=(int(bad.sum()), kmax))
        keys = np.broadcast_to(ref, (batch, W)).copy()
        for j in range(kmax):
            w = (pos[:, j] // 64).astype(np.int64)
            bit = (np.uint64(1) << (pos[:, j] % 64).astype(np.uint64))
            bit = np.where(active[:, j], bit, np.uint64(0)).astype(np.uint64)
            for ww in range(W):
                m = w == ww
                keys[m, ww] ^= bit[m]
        for row in map(bytes, keys):
            if row not in seen:
                seen.add(row)
                out.append(row)
                total += 1
                if total == count:
                    break
    buf = np.frombuffer(b"".join(out), dtype=np.uint64)
    return buf.reshape(count, W).copy()


def random_subset(keys: np.ndarray, size: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    sel = rng.choice(keys.shape[0], size=min(size, keys.shape[0]), replace=False)
    return keys[np.sort(sel)]


# -------------------------------------------------------------------- named workloads

@dataclass
class Workload:
    name: str
    ops: TermList
    keys: np.ndarray  # uint64 [n][W]


def c1_tfim12() -> Workload:
    """TFIM-12 periodic, J = h = 1, full 4096-state space."""
    return Workload("tfim12_full", tfim_chain(12, 1.0, 1.0, True), full_space(12))


def c2_xxz6x6(count: int = 1 << 20, seed: int = 2) -> Workload:
    """XXZ 6x6 open grid (Jxy = 1, Jz = 0.8, ladder form); ``count`` weight-18 strings."""
    return Workload("xxz6x6_w18_%d" % count, xxz_grid_6x6(), weight_sector_samples(36, 18, count, seed))


def c3_molecular(na: int = 1500, nb: int = 1500, seed: int = 3) -> Workload:
    """Random 16-orbital molecular Hamiltonian, 5 alpha + 5 beta electrons,
    ``na x nb`` product subspace."""
    h, eri = molecular_integrals(16, seed)
    return Workload("fermi16_%dx%d" % (na, nb), molecular_terms(h, eri),
                    product_subspace(16, 5, 5, na, nb, seed))


def c4_heavy_hex(count: int = 5_000_000, seed: int = 4) -> Workload:
    """200-qubit heavy-hex XY + Z-field model; reference 2-colouring plus 1-6 flips."""
    n, edges = heavy_hex_200()
    col = two_colouring(n, edges)
    ref = (col == 1).astype(np.uint8)
    return Workload("heavyhex200_%d" % count, heavy_hex_xy_field(),
                    reference_flip_samples(n, ref, count, seed))


def serving_requests(n_requests: int = 256, seed: int = 5, smin: float = 1e3, smax: float = 2e6):
    """Request list for the serving workload: ``(family, size, sub_seed)`` per request.

    Family is uniform over the three Hamiltonians (tfim12, xxz6x6, fermi16); size is
    log-uniform in ``[smin, smax]``."""
    rng = np.random.default_rng(seed)
    fam = rng.integers(0, 3, size=n_requests)
    size = np.floor(np.exp(rng.uniform(math.log(smin), math.log(smax), size=n_requests))).astype(np.int64)
    sub = rng.integers(0, 2**31 - 1, size=n_requests)
    out = []
    for f, s, ss in zip(fam.tolist(), size.tolist(), sub.tolist()):
        name = ("tfim12", "xxz6x6", "fermi16")[f]
        if name == "tfim12":
            s = min(s, 4096)
        out.append((name, int(s), int(ss)))
    return out


def serving_subspace(name: str, size: int, sub_seed: int) -> np.ndarray:
    if name == "tfim12":
        return random_subset(full_space(12), size, sub_seed)
    if name == "xxz6x6":
        return weight_sector_samples(36, 18, size, sub_seed, batch=max(1024, min(1 << 19, 2 * size)))
    if name == "fermi16":
        side = min(4368, int(math.ceil(math.sqrt(size))))
        return product_subspace(16, 5, 5, side, side, sub_seed)
    raise ValueError(name)
