"""Restarted GMRES (oracle; test-only).

The discretised boundary integral equations are solved matrix-free by GMRES (Sec. 4,
opening paragraphs; Saad's textbook algorithm): Arnoldi with modified Gram-Schmidt,
Givens rotations for the small least-squares problem, restart after `restart` steps.
Convergence is declared on the *true* residual ||b - A x||_2 / ||b||_2 <= tol (reading:
the paper gives no tolerance, norm or restart length).

Pinned by: agreement with a dense direct solve of the assembled matrix (columns
A e_k) at small sizes (tests/test_oracle_gmres.py).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class GmresStats:
    iters: int
    restarts: int
    applies: int
    relres: float
    converged: bool


def gmres(A, b: np.ndarray, x0: np.ndarray | None = None, tol: float = 1e-10,
          restart: int = 50, maxit: int = 1000):
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return np.zeros_like(b), GmresStats(0, 0, 0, 0.0, True)
    applies = 0
    total = 0
    restarts = 0
    while True:
        r = b - A(x)
        applies += 1
        beta = np.linalg.norm(r)
        if beta <= tol * nb or total >= maxit:
            return x, GmresStats(total, restarts, applies, beta / nb, beta <= tol * nb)
        m = restart
        V = np.zeros((m + 1, b.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gvec = np.zeros(m + 1)
        gvec[0] = beta
        V[0] = r / beta
        j_used = 0
        for j in range(m):
            w = A(V[j])
            applies += 1
            total += 1
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                           # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            j_used = j + 1
            if abs(gvec[j + 1]) <= tol * nb or total >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_used, :j_used]), gvec[:j_used])
        x = x + V[:j_used].T @ y
        restarts += 1
