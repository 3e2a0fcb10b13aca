"""CPU Lanczos ground state (FP64, full reorthogonalization).

The paper hands its matrix-free operator to an external eigensolver (Results: ARPACK via
SciPy, PRIMME LOBPCG); any converged Hermitian eigensolver reaches the same lowest
eigenvalue.  This oracle runs the textbook Lanczos three-term recurrence with full
(classical Gram-Schmidt, applied twice) reorthogonalization against all previous basis
vectors and diagonalizes the tridiagonal matrix with ``numpy.linalg.eigh`` (LAPACK).
Convergence: Ritz residual estimate ``beta_k |s_k| <= tol * |theta|``.
"""
import numpy as np


def lanczos_ground(matvec, n: int, v0=None, tol: float = 1e-12, max_iter: int = 400, dtype=np.float64):
    """Return ``(theta, ritz_vector, iterations)`` for the lowest eigenvalue."""
    if n == 1:
        x = np.ones(1, dtype=dtype)
        return float(np.real(matvec(x)[0])), x, 1
    v = np.ones(n, dtype=dtype) if v0 is None else np.asarray(v0, dtype=dtype).copy()
    v /= np.linalg.norm(v)
    V = [v]
    alphas, betas = [], []
    theta, s = None, None
    m = min(max_iter, n)
    for k in range(m):
        w = matvec(V[k]).astype(dtype)
        a = np.vdot(V[k], w).real
        w = w - a * V[k]
        if k > 0:
            w = w - betas[-1] * V[k - 1]
        Vm = np.array(V)
        for _ in range(2):
            h = Vm.conj() @ w
            w = w - Vm.T @ h
            a += h[k].real
        alphas.append(a)
        b = np.linalg.norm(w)
        T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
        ev, evec = np.linalg.eigh(T)
        theta, s = ev[0], evec[:, 0]
        if b * abs(s[-1]) <= tol * max(1.0, abs(theta)) or b < 1e-14 or k == m - 1:
            Vm = np.array(V)
            x = Vm.T @ s
            return float(theta), x / np.linalg.norm(x), k + 1
        betas.append(b)
        V.append(w / b)
    raise AssertionError("unreachable")
