"""Pure-Python double loops for tiny inputs (N <= 64).

TEST INFRASTRUCTURE ONLY (see the package docstring).  These use ``math`` on
Python floats, one entry at a time, so that the vectorised oracle can be
checked against a second, independent spelling of the same definitions
(LightGP Sec. 2 and Sec. 3 "Kernels").
"""

from __future__ import annotations

import math


def entry(family: str, xi, xj, ls, s2: float, period: float = 1.0) -> float:
    if family == "linear":
        a = 0.0
        for k in range(len(xi)):
            a += float(xi[k]) * float(xj[k])
        return s2 * a
    if family == "periodic":
        a = 0.0
        for k in range(len(xi)):
            sk = math.sin(math.pi * (float(xi[k]) - float(xj[k])) / period)
            a += 2.0 * sk * sk / (float(ls[k]) * float(ls[k]))
        return s2 * math.exp(-a)
    r2 = 0.0
    for k in range(len(xi)):
        t = (float(xi[k]) - float(xj[k])) / float(ls[k])
        r2 += t * t
    rho = math.sqrt(r2)
    if family == "rbf":
        return s2 * math.exp(-r2 / 2.0)
    if family == "matern12":
        return s2 * math.exp(-rho)
    if family == "matern32":
        a = math.sqrt(3.0) * rho
        return s2 * (1.0 + a) * math.exp(-a)
    if family == "matern52":
        a = math.sqrt(5.0) * rho
        return s2 * (1.0 + a + a * a / 3.0) * math.exp(-a)
    raise ValueError(family)


def ky_matvec(family, X, V, ls, s2, noise):
    """out[i][c] = sum_j k(x_i, x_j) V[j][c] + noise V[i][c] with nested loops."""
    n = len(X)
    t = len(V[0])
    out = [[0.0] * t for _ in range(n)]
    for i in range(n):
        for j in range(n):
            k = entry(family, X[i], X[j], ls, s2)
            for c in range(t):
                out[i][c] += k * float(V[j][c])
        for c in range(t):
            out[i][c] += noise * float(V[i][c])
    return out


def gauss_solve(A, b):
    """Gaussian elimination with partial pivoting on lists (tiny SPD systems)."""
    n = len(A)
    M = [list(map(float, A[i])) + [float(b[i])] for i in range(n)]
    for col in range(n):
        piv = max(range(col, n), key=lambda r: abs(M[r][col]))
        M[col], M[piv] = M[piv], M[col]
        for r in range(col + 1, n):
            f = M[r][col] / M[col][col]
            for c in range(col, n + 1):
                M[r][c] -= f * M[col][c]
    x = [0.0] * n
    for r in range(n - 1, -1, -1):
        s = M[r][n] - sum(M[r][c] * x[c] for c in range(r + 1, n))
        x[r] = s / M[r][r]
    return x


def log_det(A):
    """log det of a small SPD matrix by elimination without pivoting."""
    n = len(A)
    M = [list(map(float, row)) for row in A]
    acc = 0.0
    for col in range(n):
        acc += math.log(M[col][col])
        for r in range(col + 1, n):
            f = M[r][col] / M[col][col]
            for c in range(col, n):
                M[r][c] -= f * M[col][c]
    return acc


def mll(family, X, y, ls, s2, noise):
    n = len(X)
    A = [[entry(family, X[i], X[j], ls, s2) + (noise if i == j else 0.0) for j in range(n)]
         for i in range(n)]
    a = gauss_solve(A, y)
    quad = sum(float(y[i]) * a[i] for i in range(n))
    return -0.5 * (quad + log_det(A) + n * math.log(2.0 * math.pi))
