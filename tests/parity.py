"""Comparison helpers of the GPU parity tests: relative l2 error over the whole vector and
largest elementwise error relative to the largest reference entry, both held to the same
tolerance (a localized error is then not diluted by the rest of the vector)."""
import numpy as np


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def check(got, want, tol, what=""):
    """Assert rel(got, want) <= tol and maxrel(got, want) <= tol, or, with tol a pair
    (l2, max), each bound on its own measure; returns both errors."""
    t2, tm = tol if isinstance(tol, tuple) else (tol, tol)
    e2, em = rel(got, want), maxrel(got, want)
    print(f"  {what}: rel {e2:.3e} max {em:.3e}")
    assert e2 <= t2 and em <= tm, (what, e2, em, tol)
    return e2, em


# FP32 grid stages against the FP64 oracle, (relative l2, largest element relative to the
# largest reference entry), about five times the largest errors measured over the parity
# cases (1024^2 and 2048^2 stars, Laplace and modified Helmholtz, zero, free-space and
# zero-normal-derivative boxes): traces 9e-7 and 2.2e-6; normal derivatives 1.5e-5 and
# 6.4e-5 (the normal derivative differences grid values over h, so its FP32 error grows
# like 1/h).
TOL32 = {"v_plus": (5e-6, 1.2e-5), "v_minus": (5e-6, 1.2e-5),
         "dn_plus": (8e-5, 3.2e-4), "dn_minus": (8e-5, 3.2e-4)}
