"""Exact rational GN on tiny integer inputs (brute-force pin for the FP64 oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

With integer A, X, Y and a core C = Y^T A X of full column rank, the
pseudoinverse is C^+ = (C^T C)^{-1} C^T (Section 2: the definition of the
pseudoinverse, specialised to full column rank), and the plain GN approximant
AX C^+ Y^T A (Section 2, eq. (3)) is a matrix of rationals computed here without
rounding, by Gauss-Jordan elimination over fractions.Fraction.
"""
from __future__ import annotations

from fractions import Fraction


def _mat(a):
    return [[Fraction(int(v)) if not isinstance(v, Fraction) else v for v in row] for row in a]


def matmul(A, B):
    n, k, m = len(A), len(B), len(B[0])
    return [[sum((A[i][t] * B[t][j] for t in range(k)), Fraction(0)) for j in range(m)]
            for i in range(n)]


def transpose(A):
    return [list(col) for col in zip(*A)]


def inverse(M):
    """Inverse of a square rational matrix by Gauss-Jordan elimination."""
    n = len(M)
    aug = [list(M[i]) + [Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for c in range(n):
        p = next(i for i in range(c, n) if aug[i][c] != 0)    # singular -> StopIteration
        aug[c], aug[p] = aug[p], aug[c]
        piv = aug[c][c]
        aug[c] = [v / piv for v in aug[c]]
        for i in range(n):
            if i != c and aug[i][c] != 0:
                f = aug[i][c]
                aug[i] = [a - f * b for a, b in zip(aug[i], aug[c])]
    return [row[n:] for row in aug]


def gn_exact(A, X, Y):
    """Exact AX (Y^T A X)^+ Y^T A for integer matrices, C of full column rank."""
    A, X, Y = _mat(A), _mat(X), _mat(Y)
    AX = matmul(A, X)
    YT = transpose(Y)
    YA = matmul(YT, A)
    C = matmul(YT, AX)
    CT = transpose(C)
    Cp = matmul(inverse(matmul(CT, C)), CT)
    return matmul(matmul(AX, Cp), YA)
