"""Alternative stabilizations of the GN core and the plain-GN instability check,
FP64 on the CPU (Section 5.1.1 and Section 5.1.2).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Section 5.1.1 lists, besides the truncated QR used by oracle.gn.core:
  * the SVD route: take the SVD of the core C = Y^T A X, drop the singular values
    below the threshold and apply the pseudoinverse of what is left
    (core_svd / factors_svd);
  * three perturbations that make every singular value of the core at least the
    threshold instead of truncating, so that the inverse of the triangular (or
    diagonal) factor is bounded by one over the threshold:
      (a) lift the small singular values of the SVD             -- lift_svd
      (b) lift the small diagonal entries of R from a rank-revealing QR (here
          Householder QR with column pivoting, C P = Q R)       -- lift_rrqr
      (c) lift the small diagonal entries of the unpivoted R     -- lift_diag
    (a) and (b) bound the inverse by construction when the factorization reveals
    the rank; (c) is expected to with high probability for random sketches but
    can fail on adversarial triangular factors (Kahan's matrix).
Section 5.1.2 checks plain GN with a power-method estimate of the 2-norm of the
inverse triangular factor (two triangular solves per step, O(r^2)), and switches
to SGN only when the estimate exceeds one over the threshold (inv_norm_power,
check, gn_checked).

Readings where the paper leaves a choice open: the threshold is the same tau = eps nu_X
nu_Y as the truncated QR; a kept singular value is one >= tau (ties go to the
kept side, as for R's diagonal); a lifted value is set to tau (with the sign of
the diagonal entry it replaces, + for zero); the power method runs on a block of
start vectors drawn from Philox stream 6 (the first k entries of each row of an
nv x r block) and reports the largest ||T^{-T} x|| over unit iterates x, a lower
bound of ||T^{-1}||_2, with T the factor whose inverse multiplies AX (R, or R_2^T
when truncated); the check flags when
estimate * delta * nu_X * nu_Y > 1, i.e. when plain GN's triangular factor has a
singular value below the threshold that eps = delta would use.

Pins (tests/test_oracle_stabilize.py): closed forms on cores built from chosen
singular values and vectors; plain GN when nothing is below the threshold; exact
recovery of a rank-deficient matrix; the column-pivoted QR's defining properties;
the bound on the inverse after (a) and (b) and its failure for (c) on Kahan's
matrix; the power method's lower-bound property against the exact norm and its
convergence on matrices with a gap; the check's decision on both sides of the
threshold.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import philox
from .gn import _qr_nonneg


@dataclass
class Factored:
    """A_hat = F G with F = AX B (m x k) and G = L (Y^T A) (k x n)."""
    F: np.ndarray
    G: np.ndarray
    k: int              # kept rank (r for the perturbations)
    lifted: int         # entries raised to the threshold (perturbations only)
    values: np.ndarray  # singular values of C, or R's diagonal, before lifting
    status: int = 0     # 1 non-finite core, 2 nothing kept

    @property
    def approx(self) -> np.ndarray:
        return self.F @ self.G


def _finite_or_status(C):
    return 0 if np.all(np.isfinite(C)) else 1


def core_matrix(AX: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """C = Y^T (AX), the order of the Section 5.1 evaluation."""
    return Y.T @ AX


# ----------------------------------------------------------------------------- SVD route
def core_svd(AX, YA, Y, tau: float) -> Factored:
    """SGN through the SVD of C: keep sigma_i >= tau (tau <= 0: sigma_i > 0),
    F = AX V_k diag(1/sigma_k), G = U_k^T (Y^T A)  (Section 5.1.1, first option)."""
    C = core_matrix(AX, Y)
    if _finite_or_status(C):
        r = C.shape[1]
        return Factored(np.zeros((AX.shape[0], 0)), np.zeros((0, YA.shape[1])), 0, 0,
                        np.full(r, np.nan), 1)
    U, s, Vt = np.linalg.svd(C, full_matrices=False)
    keep = (s >= tau) if tau > 0 else (s > 0)
    k = int(np.argmin(keep)) if not keep.all() else len(s)   # s is sorted: a prefix
    F = (AX @ Vt[:k].T) / s[:k]
    G = U[:, :k].T @ YA
    return Factored(F, G, k, 0, s, 0 if k > 0 else 2)


def lift_svd(AX, YA, Y, tau: float) -> Factored:
    """Perturbation (a): singular values below tau raised to tau, nothing dropped."""
    C = core_matrix(AX, Y)
    U, s, Vt = np.linalg.svd(C, full_matrices=False)
    sl = np.maximum(s, tau)
    F = (AX @ Vt.T) / sl
    G = U.T @ YA
    return Factored(F, G, len(s), int(np.sum(s < tau)), s)


# ----------------------------------------------------------------------------- QR routes
def _lift_diagonal(R: np.ndarray, tau: float):
    """R with every |R_ii| < tau replaced by tau carrying R_ii's sign (+ for 0)."""
    R = R.copy()
    d = np.diag(R).copy()
    low = np.abs(d) < tau
    d[low] = np.where(d[low] < 0, -tau, tau)
    R[np.diag_indices_from(R)] = d
    return R, int(np.sum(low))


def qr_pivoted(C: np.ndarray):
    """Householder QR with column pivoting (Businger-Golub; LAPACK geqp3):
    C[:, p] = Q R with |R_11| >= |R_22| >= ... ."""
    Q, R, p = sla.qr(C, mode="economic", pivoting=True)
    return Q, R, p


def lift_rrqr(AX, YA, Y, tau: float) -> Factored:
    """Perturbation (b): C P = Q R by column-pivoted QR, small |R_ii| raised to tau;
    A_hat = (AX P) R'^{-1} (Q^T (Y^T A))."""
    C = core_matrix(AX, Y)
    Q, R, p = qr_pivoted(C)
    Rl, lifted = _lift_diagonal(R, tau)
    F = sla.solve_triangular(Rl, AX[:, p].T, trans="T", lower=False).T
    G = Q.T @ YA
    return Factored(F, G, R.shape[0], lifted, np.diag(R).copy())


def lift_diag(AX, YA, Y, tau: float) -> Factored:
    """Perturbation (c): the unpivoted R (diagonal >= 0) with R_ii < tau raised to
    tau; A_hat = (AX R'^{-1}) (Q^T (Y^T A))."""
    C = core_matrix(AX, Y)
    Q, R = _qr_nonneg(C)
    Rl, lifted = _lift_diagonal(R, tau)
    F = sla.solve_triangular(Rl, AX.T, trans="T", lower=False).T
    G = Q.T @ YA
    return Factored(F, G, R.shape[0], lifted, np.diag(R).copy())


# ----------------------------------------------------------------------------- Section 5.1.2
def power_start(seed: int, nv: int, k: int) -> np.ndarray:
    """Start vectors of the power method: rows of a Gaussian block on stream 6."""
    return philox.gaussian(seed, philox.STREAM_POWER, nv, k)


def inv_norm_power(T: np.ndarray, V0: np.ndarray, iters: int, lower: bool = False) -> float:
    """Power-method estimate of ||T^{-1}||_2 for triangular T (k x k).

    Each row v of V0 is normalized, then per step y = T^{-T} v and z = T^{-1} y by
    substitution (O(k^2)); the estimate is the largest ||y|| seen, a lower bound
    of ||T^{-1}||_2 = sqrt(lambda_max((T T^T)^{-1})); v <- z / ||z||."""
    k = T.shape[0]
    if k == 0 or V0.shape[0] == 0:
        return 0.0
    V = V0 / np.linalg.norm(V0, axis=1, keepdims=True)
    est = 0.0
    for _ in range(iters):
        Yv = sla.solve_triangular(T, V.T, trans="T", lower=lower)   # columns y_i
        est = max(est, float(np.max(np.linalg.norm(Yv, axis=0))))
        Z = sla.solve_triangular(T, Yv, trans="N", lower=lower)
        V = (Z / np.linalg.norm(Z, axis=0, keepdims=True)).T
    return est


def applied_triangle(c):
    """(T, lower): the triangular factor whose inverse the factor application
    applies to AX, for an oracle.gn.Core: T = R when k == r (F = AX R^{-1}) and
    T = R_2^T when k < r (F = (AX Q_2) R_2^{-T}); ||R_2^{-1}|| = ||R_1^+||."""
    if c.k == c.R.shape[0]:
        return c.R, False
    return c.R2.T, True


def check(c, delta: float, nu_x: float, nu_y: float, seed: int, nv: int = 8, iters: int = 4):
    """Section 5.1.2: (estimate, flag) with flag = estimate * delta nu_x nu_y > 1."""
    T, lower = applied_triangle(c)
    est = inv_norm_power(T, power_start(seed, nv, T.shape[0]), iters, lower)
    return est, bool(est * delta * nu_x * nu_y > 1.0)


def gn_checked(A, X, Y, delta: float, nu_x: float, nu_y: float, seed: int, nv: int = 8,
               iters: int = 4):
    """Plain GN, checked; SGN with eps = delta (truncated QR) only when flagged.
    Returns (GNResult, estimate, flagged)."""
    from . import gn as G
    res = G.gn(A, X, Y, 0.0)
    est, flag = check(res.core, delta, nu_x, nu_y, seed, nv, iters)
    if flag:
        res = G.gn(A, X, Y, G.threshold(delta, nu_x, nu_y))
    return res, est, flag
