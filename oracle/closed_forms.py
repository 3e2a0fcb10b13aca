"""Textbook ground energies used to pin the oracle (and, through it, the GPU path).

* Periodic transverse-field Ising chain ``H = -J sum Z_i Z_{i+1} - h sum X_i`` with even
  ``L``: the ground state lies in the even-parity (Neveu-Schwarz) sector of the free-fermion
  solution, ``E0 = -sum_{m=1}^{L} sqrt(J^2 + h^2 - 2 J h cos(pi (2m-1) / L))``; at
  ``J = h = 1`` this is ``-2 / sin(pi / (2L))``.
* Open XY chain with a field ``H = sum J (X_i X_{i+1} + Y_i Y_{i+1}) + h sum Z_i``: with
  ``|1>`` occupied, ``Z = 1 - 2n`` and ``XX + YY = 2 (c+ c + h.c.)``, giving single-particle
  energies ``4 J cos(pi k / (L+1)) - 2 h`` and ``E0 = h L + sum_k min(0, e_k)``.
* Quadratic fermions ``sum h_pq f+_p f_q`` in the ``N``-particle sector: the sum of the ``N``
  lowest eigenvalues of ``h``.
* Commuting one- and two-body terms: with ``h = V diag(eps) V^T`` and
  ``(pq|rs) = u_pq u_rs``, ``u = V diag(lam) V^T``, the chemists'-notation Hamiltonian
  ``sum h_pq f+_p f_q + 1/2 sum (pq|rs) f+_p f+_r f_s f_q`` has eigenvalues
  ``sum_{k in occ} eps_k + sum_{k<l in occ} lam_k lam_l`` on Slater determinants of the
  columns of ``V`` (because ``1/2 sum u_pq u_rs f+_p f+_r f_s f_q = 1/2 (U^2 - sum (u^2)_ps
  f+_p f_s)`` with ``U = sum u_pq f+_p f_q``); the ground energy is the minimum over
  ``N``-subsets.
"""
from itertools import combinations
import math

import numpy as np


def tfim_periodic_e0(L: int, J: float = 1.0, h: float = 1.0) -> float:
    assert L % 2 == 0
    return -sum(math.sqrt(J * J + h * h - 2 * J * h * math.cos(math.pi * (2 * m - 1) / L)) for m in range(1, L + 1))


def xy_open_field_e0(L: int, J: float, h: float) -> float:
    e = [4 * J * math.cos(math.pi * k / (L + 1)) - 2 * h for k in range(1, L + 1)]
    return h * L + sum(min(0.0, x) for x in e)


def quadratic_fermion_e0(h: np.ndarray, n_particles: int) -> float:
    ev = np.linalg.eigvalsh(h)
    return float(np.sum(ev[:n_particles]))


def commuting_two_body_e0(eps: np.ndarray, lam: np.ndarray, n_particles: int) -> float:
    best = math.inf
    for occ in combinations(range(len(eps)), n_particles):
        e = sum(eps[k] for k in occ)
        for a in range(len(occ)):
            for b in range(a + 1, len(occ)):
                e += lam[occ[a]] * lam[occ[b]]
        best = min(best, e)
    return float(best)


def commuting_two_body_e0_spin(eps: np.ndarray, lam: np.ndarray, n_alpha: int, n_beta: int) -> float:
    """Spinful version: the two-body operator couples every pair of occupied spin orbitals
    (``sum_{sigma,tau}``), so the eigenvalue of a determinant with alpha set ``A`` and beta set
    ``B`` is ``sum_{A} eps + sum_{B} eps + sum_{pairs in A+B} lam lam``."""
    norb = len(eps)
    best = math.inf
    for A in combinations(range(norb), n_alpha):
        for B in combinations(range(norb), n_beta):
            occ = [lam[k] for k in A] + [lam[k] for k in B]
            e = sum(eps[k] for k in A) + sum(eps[k] for k in B)
            s = sum(occ)
            e += 0.5 * (s * s - sum(x * x for x in occ))
            best = min(best, e)
    return float(best)
