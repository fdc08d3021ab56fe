"""Reverse mode of the (S)GN approximant, FP64 on the CPU.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper defines the forward map only; differentiating it is an extension of
the method.  What is differentiated is the approximant of Section 5.1.1 with the
kept rank k held at the value the forward pass chose:

    P = AX,  S = Y^T A,  C = Y^T P,            (Algorithm 2.1, steps 1-2)
    C = Q R (Householder, R_ii >= 0),  Q_1 = Q[:, :k],  R_1 = R[:k, :]
    M = R_1^+ Q_1^T   (= R^-1 Q^T when k = r; = Q_2 R_2^{-T} Q_1^T when k < r,
                       with R_1^T = Q_2 R_2)   (Section 5.1.1)
    A_hat = P M S,    L = <Gbar, A_hat>.

With k fixed, M is the pseudoinverse of the rank-k matrix B = P_1 C, where P_1 =
Q_1 Q_1^T is the orthogonal projector onto the span of the first k columns of C
(the Householder QR without pivoting orthogonalizes the columns in order).  The
chain rule then needs two classical derivatives:

  * the pseudoinverse of a matrix of constant rank (Golub and Pereyra, 1973):
        dM = -M dB M + M M^T dB^T (I - B M) + (I - M B) dB^T M^T M,
    whose adjoint, for H = dL/dM, is
        Bbar = -M^T H M^T + (I - B M) H^T M M^T + M^T M H^T (I - M B);
  * the projector onto the span of C_1 = C[:, :k] (full column rank):
        dP_1 = (I - P_1) dC_1 C_1^+ + (C_1^+)^T dC_1^T (I - P_1),
    with adjoint, for Pbar = dL/dP_1,  C_1bar = (I - P_1)(Pbar + Pbar^T)(C_1^+)^T,
    and (C_1^+)^T = Q_1 R_11^{-T}.

Collecting terms (G1 = Gbar S^T, G2 = P^T Gbar, H = P^T G1):

    Cbar = P_1 Bbar + [ (I - P_1)(Bbar C^T + C Bbar^T) Q_1 R_11^{-T} , 0 ]
    dL/dA = G1 M^T X^T + Y M^T G2 + Y Cbar X^T.

Pins (tests/test_oracle_grad.py): central finite differences of L in FP64, with k
held fixed, in random directions and entry by entry, for k = r and k < r; and an
independent reverse-mode reference, torch's FP64 autograd through a plain torch
forward of the same map (its own QR and linear-solve adjoints).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .gn import Core, _qr_nonneg


def core_pinv(c: Core) -> np.ndarray:
    """M = R_1^+ Q_1^T (r x (r+l)), the truncated core pseudoinverse (Sec. 5.1.1)."""
    k, r = c.k, c.R.shape[0]
    Q1 = c.Q[:, :k]
    if k == r:
        return sla.solve_triangular(c.R, Q1.T, lower=False)
    return c.Q2 @ sla.solve_triangular(c.R2, Q1.T, trans="T", lower=False)


def approx_fixed_rank(A: np.ndarray, X: np.ndarray, Y: np.ndarray, k: int) -> np.ndarray:
    """A_hat = (AX) M (Y^T A) with the kept rank forced to k (the map whose
    derivative gn_backward returns)."""
    P, S = A @ X, Y.T @ A
    C = Y.T @ P
    r = C.shape[1]
    Q, R = _qr_nonneg(C)
    if k == r:
        M = sla.solve_triangular(R, Q.T, lower=False)
    else:
        Q2, R2 = _qr_nonneg(R[:k, :].T)
        M = Q2 @ sla.solve_triangular(R2, Q[:, :k].T, trans="T", lower=False)
    return P @ M @ S


def loss_fixed_rank(A, X, Y, k: int, Gbar) -> float:
    """L = <Gbar, A_hat> with the kept rank held at k."""
    return float(np.sum(Gbar * approx_fixed_rank(A, X, Y, k)))


def gn_backward(A: np.ndarray, X: np.ndarray, Y: np.ndarray, c: Core, Gbar: np.ndarray,
                AX: np.ndarray | None = None, YA: np.ndarray | None = None) -> np.ndarray:
    """dL/dA for L = <Gbar, A_hat>, A_hat the (S)GN approximant of the forward pass
    described by the core `c` (its k held fixed).  Returns an m x n FP64 array."""
    P = A @ X if AX is None else AX
    S = Y.T @ A if YA is None else YA
    k = c.k
    rl = c.Q.shape[0]
    M = core_pinv(c)                      # r x rl
    Q1 = c.Q[:, :k]
    C = c.C
    G1 = Gbar @ S.T                       # m x rl
    G2 = P.T @ Gbar                       # r x n
    H = P.T @ G1                          # r x rl  = dL/dM
    P1 = Q1 @ Q1.T                        # B M
    MB = M @ (Q1 @ c.R[:k, :])            # M B  (projector onto the row space of R_1)
    I_rl = np.eye(rl)
    I_r = np.eye(M.shape[0])
    Bbar = (-M.T @ H @ M.T + (I_rl - P1) @ H.T @ (M @ M.T)
            + (M.T @ M) @ H.T @ (I_r - MB))
    Cbar = P1 @ Bbar
    C1pT = sla.solve_triangular(c.R[:k, :k], Q1.T, lower=False).T  # (R_11^-1 Q_1^T)^T
    Pbar = Bbar @ C.T
    Cbar[:, :k] += (I_rl - P1) @ (Pbar + Pbar.T) @ C1pT
    return G1 @ M.T @ X.T + Y @ (M.T @ G2) + Y @ Cbar @ X.T
