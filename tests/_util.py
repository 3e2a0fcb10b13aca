"""Shared helpers for the GPU parity tests (inputs and oracle calls only)."""
import functools
import sys

import numpy as np

import workloads as wl
from oracle import rowwise as orw
from oracle import subspace as osub


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dyadic(tl: wl.TermList, bits: int = 20) -> wl.TermList:
    """Same structure, coefficients rounded to multiples of 2^-bits (zeros bumped to one unit),
    so that every sum the method forms is exact in FP64 whatever its order."""
    s = float(1 << bits)
    re = np.round(tl.coef.real * s)
    im = np.round(tl.coef.imag * s)
    re[(re == 0) & (im == 0)] = 1.0
    return wl.TermList(tl.n_qubits, tl.term_ptr, tl.op_idx, tl.op_code, (re + 1j * im) / s, tl.fermionic)


def dyadic_vector(rng, n, bits: int = 10, nvec: int = 1, dtype=np.float64):
    k = rng.integers(-(1 << bits) + 1, 1 << bits, size=(n, nvec))
    v = (k / float(1 << bits)).astype(dtype)
    return v[:, 0] if nvec == 1 else v


@functools.lru_cache(maxsize=None)
def c2_keys(count: int):
    return wl.c2_xxz6x6(count).keys


@functools.lru_cache(maxsize=None)
def c3_parts(na: int, nb: int):
    w = wl.c3_molecular(na, nb)
    return w.ops, w.keys


def oracle_csr_rows(keys, tl, rows=None):
    ck = osub.canonical_keys(keys)
    return ck, orw.rows_c(ck, tl, rows)


def heavy_hex_small(count: int, seed: int = 4):
    n, edges = wl.heavy_hex_200()
    col = wl.two_colouring(n, edges)
    ref = (col == 1).astype(np.uint8)
    return wl.heavy_hex_xy_field(), wl.reference_flip_samples(n, ref, count, seed, batch=1 << 16)
