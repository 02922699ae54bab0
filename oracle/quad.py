"""1D building blocks: Jacobi polynomials, Gauss rules, Lagrange polynomials.

Gauss-Jacobi rules come from ``scipy.special.roots_jacobi`` (weight
(1-x)^alpha (1+x)^beta on [-1,1]); Jacobi polynomial values from
``scipy.special.eval_jacobi``.  Derivatives use
d/dx P_n^{(a,b)} = (n+a+b+1)/2 P_{n-1}^{(a+1,b+1)}.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def jacobi(n: int, a: float, b: float, x):
    """Unnormalised Jacobi polynomial P_n^{(a,b)}(x)."""
    x = np.asarray(x, dtype=np.float64)
    if n < 0:
        return np.zeros_like(x)
    return special.eval_jacobi(n, a, b, x)


def djacobi(n: int, a: float, b: float, x):
    """Derivative of P_n^{(a,b)} at x."""
    x = np.asarray(x, dtype=np.float64)
    if n <= 0:
        return np.zeros_like(x)
    return 0.5 * (n + a + b + 1.0) * special.eval_jacobi(n - 1, a + 1.0, b + 1.0, x)


def gauss_jacobi(n: int, a: float = 0.0, b: float = 0.0):
    """n-point Gauss-Jacobi rule for weight (1-x)^a (1+x)^b; nodes ascending."""
    x, w = special.roots_jacobi(n, a, b)
    order = np.argsort(x)
    return np.asarray(x[order], dtype=np.float64), np.asarray(w[order], dtype=np.float64)


def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule (exact to degree 2n-1)."""
    return gauss_jacobi(n, 0.0, 0.0)


def gauss_lobatto(n: int):
    """n-point Gauss-Legendre-Lobatto rule (n >= 2): +-1 and the roots of P'_{n-1}."""
    N = n - 1
    if N == 1:
        return np.array([-1.0, 1.0]), np.array([1.0, 1.0])
    xi, _ = gauss_jacobi(N - 1, 1.0, 1.0)
    x = np.concatenate([[-1.0], xi, [1.0]])
    w = 2.0 / (N * (N + 1) * jacobi(N, 0.0, 0.0, x) ** 2)
    return x, w


def lagrange(nodes, y):
    """Values L[m, j] = l_j(y_m) of the Lagrange polynomials on ``nodes``."""
    nodes = np.asarray(nodes, dtype=np.float64)
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    n = nodes.size
    L = np.ones((y.size, n))
    for j in range(n):
        for m in range(n):
            if m != j:
                L[:, j] *= (y - nodes[m]) / (nodes[j] - nodes[m])
    return L


def dlagrange(nodes, y):
    """Derivatives D[m, j] = l_j'(y_m), by the product rule."""
    nodes = np.asarray(nodes, dtype=np.float64)
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    n = nodes.size
    D = np.zeros((y.size, n))
    for j in range(n):
        for k in range(n):
            if k == j:
                continue
            term = np.full(y.size, 1.0 / (nodes[j] - nodes[k]))
            for m in range(n):
                if m != j and m != k:
                    term *= (y - nodes[m]) / (nodes[j] - nodes[m])
            D[:, j] += term
    return D
