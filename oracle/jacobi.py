"""Plain cyclic two-sided Jacobi for small Hermitian matrices (TEST INFRASTRUCTURE).

An independent cross-check of LAPACK ``eigh`` for the EVD of Eq. 2: each
off-diagonal entry (p, q) is removed by a unitary plane rotation built from the
2x2 Hermitian block, first rotating away the phase of a_pq, then applying the
classical real Jacobi rotation. Pure Python loops: use for n <= 32 only.
"""
from __future__ import annotations

import math

import numpy as np


def jacobi_eigh(a: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Return (eigenvalues descending, eigenvectors as columns, sweeps used)."""
    a = np.array(a, dtype=np.complex128)
    n = a.shape[0]
    v = np.eye(n, dtype=np.complex128)
    scale = np.linalg.norm(a)
    sweeps = 0
    for sweeps in range(1, max_sweeps + 1):
        off = float(np.linalg.norm(a - np.diag(np.diag(a))))
        if off <= tol * scale:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = a[p, q]
                mag = abs(apq)
                if mag == 0.0:
                    continue
                phase = apq / mag
                theta = (a[q, q].real - a[p, p].real) / (2.0 * mag)
                t = (1.0 if theta >= 0 else -1.0) / (abs(theta) + math.sqrt(theta * theta + 1.0))
                c = 1.0 / math.sqrt(t * t + 1.0)
                s = t * c
                # J = diag(1, conj(phase)) @ [[c, s], [-s, c]]
                j = np.array([[c, s], [-s * phase.conjugate(), c * phase.conjugate()]])
                cols = [p, q]
                a[:, cols] = a[:, cols] @ j
                a[cols, :] = j.conj().T @ a[cols, :]
                v[:, cols] = v[:, cols] @ j
    lam = np.real(np.diag(a))
    order = np.argsort(-lam, kind="stable")
    return lam[order], v[:, order], sweeps
