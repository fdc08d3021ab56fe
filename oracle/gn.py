"""Generalized Nystrom (GN) and stabilized GN (SGN), FP64 on the CPU.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

What is computed, and where the paper defines it:
  * plain GN, A_hat = AX (Y^T A X)^+ Y^T A                 -- Section 2, eq. (3)
  * SGN, A_hat = AX (Y^T A X)_eps^+ Y^T A, where (.)_eps^+ keeps singular values
    above eps                                             -- Section 2, eq. (4)
  * the pipeline: sketches X (n x r), Y (m x (r+l)), l = ceil(r/2); AX and Y^T A;
    QR of Y^T A X; A_hat = ((AX) R^-1)(Q^T (Y^T A))       -- Algorithm 2.1
  * the stable evaluation order (QR of Y^T (AX), triangular solve on AX, never an
    explicit R^-1 Q^T or pinv of the core)                -- Section 5.1
  * SGN by truncated QR: drop the trailing rows of R whose diagonal falls below
    the threshold, R_1 = R[:k, :], QR(R_1^T) = Q_2 R_2, core pseudoinverse
    Q_2 R_2^{-T} Q_1^T                                    -- Section 5.1.1
  * products with the factors, A_hat W = AX(R^-1(Q^T(Y^T A W))) and
    W A_hat = (((W AX) R^-1) Q^T) Y^T A                   -- Section 2, after Alg. 2.1

Readings taken where the paper is silent or garbled:
  * the core is formed as Y^T (AX) (the order of the Section 5.1 MATLAB line);
    core_right forms it as (Y^T A) X, the order Section 2.3 counts;
  * Householder QR without pivoting; R's diagonal made non-negative by flipping
    the matching columns of Q (the approximant does not depend on it);
  * truncation threshold tau = eps * nu_X * nu_Y on |R_ii|, with nu the sketch
    norm scale (sqrt(rows) + sqrt(cols) for Gaussians, Section 3.1; sqrt(n') for
    +-1 SRHT columns); k is the first index with |R_ii| < tau (prefix rule);
  * Section 5.1.1 prints Q_2 R_2^{-1} Q_1^T; since R_1 = R_2^T Q_2^T the
    pseudoinverse of R_1 is Q_2 R_2^{-T}, which is what is used here.

Comparison formulas used only as pins: HMT (Algorithm 1.1), Tropp17
(Section 2.4: Q (Y^T Q)^+ Y^T A with AX = QR), the SVD epsilon-pseudoinverse
(Section 2 definition; Section 5.1.1 first option), Nystrom (Section 1, eq. (1)),
CUR with identity-column sketches (Section 2.4.1), and the expectation bounds of
Theorems 3.1 and 3.2.

Every function here is pinned by a CPU test (exact recovery, the integer
truncation rank, the theorem bounds, equality with Tropp17, SVD, Nystrom, HMT and
CUR special cases, exact rational arithmetic on tiny inputs, scaling invariance,
the interpolation property); see tests/test_oracle_pins.py.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import philox


# ----------------------------------------------------------------------------- parameters
def default_l(r: int) -> int:
    """Oversampling l = ceil(r/2) (Algorithm 2.1 step 1; Section 5.2)."""
    return (r + 1) // 2


def nu_gaussian(rows: int, cols: int) -> float:
    """Upper edge of the singular values of a rows x cols Gaussian (Section 3.1)."""
    return math.sqrt(rows) + math.sqrt(cols)


def nu_srht(n: int) -> float:
    """2-norm of a +-1 SRHT sketch built from H of order n' = next pow2 >= n."""
    return math.sqrt(philox.next_pow2(n))


def threshold(eps: float, nu_x: float, nu_y: float) -> float:
    return eps * nu_x * nu_y


# ----------------------------------------------------------------------------- sketches
def gaussian_sketches(seed: int, m: int, n: int, r: int, l: int, mode: str = "f64",
                      workers: int = 1):
    """X (n x r) on stream 1 and Y (m x (r+l)) on stream 2, as FP64 arrays holding
    the values of the working precision ("f64", "f32" or "bf16").  `workers`
    host threads draw blocks of rows (same values)."""
    X = philox.gaussian(seed, philox.STREAM_X, n, r, workers=workers)
    Y = philox.gaussian(seed, philox.STREAM_Y, m, r + l, workers=workers)
    return round_mode(X, mode), round_mode(Y, mode)


def round_mode(x: np.ndarray, mode: str) -> np.ndarray:
    if mode == "f64":
        return x
    if mode == "f32":
        return philox.round_fp32(x).astype(np.float64)
    if mode == "bf16":
        return philox.round_bf16(x)
    if mode == "f16":
        return philox.round_f16(x)
    raise ValueError(mode)


def block_scales(A: np.ndarray, block: int = 128) -> np.ndarray:
    """s = 2**ceil(log2 max|a|) for each block x block tile of A (1 for an
    all-zero tile), as FP64 ceil(m/block) x ceil(n/block)."""
    A = np.asarray(A, np.float64)
    m, n = A.shape
    mb, nb = -(-m // block), -(-n // block)
    scales = np.ones((mb, nb), np.float64)
    for bi in range(mb):
        for bj in range(nb):
            t = A[bi * block:(bi + 1) * block, bj * block:(bj + 1) * block]
            mx = float(np.max(np.abs(t))) if t.size else 0.0
            if mx > 0.0:
                f, e = math.frexp(mx)          # mx = f * 2**e, f in [0.5, 1)
                scales[bi, bj] = math.ldexp(1.0, e - 1 if f == 0.5 else e)
    return scales


def block_quantize_f16(A: np.ndarray, block: int = 128):
    """Per-block power-of-two scaling and IEEE binary16 storage of A: the scales
    of block_scales and the stored value RNE_binary16(a / s).  Returns (bits
    uint16 m x n, scales float32).  The scale puts each block's largest entry in
    [0.5, 1], so entries down to 2^-14 of it stay out of the subnormal range."""
    A = np.asarray(A, np.float64)
    m, n = A.shape
    scales = block_scales(A, block)
    s_full = np.repeat(np.repeat(scales, block, 0), block, 1)[:m, :n]
    bits = (A / s_full).astype(np.float16).view(np.uint16)
    return bits, scales.astype(np.float32)


def block_dequantize_f16(bits: np.ndarray, scales: np.ndarray, block: int = 128):
    m, n = bits.shape
    s_full = np.repeat(np.repeat(scales.astype(np.float64), block, 0), block, 1)[:m, :n]
    return np.asarray(bits, np.uint16).view(np.float16).astype(np.float64) * s_full


def block_quantize_bf16(A: np.ndarray, block: int = 128):
    """Per-block power-of-two scaling and bfloat16 storage of A.

    For each block x block tile, s = 2**ceil(log2 max|a|) (s = 1 for an all-zero
    tile) and the stored value is RNE_bf16(a / s).  Returns (bits uint16 m x n,
    scales float32 ceil(m/block) x ceil(n/block)).  Power-of-two scales keep the
    division exact.
    """
    A = np.asarray(A, np.float64)
    m, n = A.shape
    mb, nb = -(-m // block), -(-n // block)
    scales = np.ones((mb, nb), np.float64)
    for bi in range(mb):
        for bj in range(nb):
            t = A[bi * block:(bi + 1) * block, bj * block:(bj + 1) * block]
            mx = float(np.max(np.abs(t))) if t.size else 0.0
            if mx > 0.0:
                f, e = math.frexp(mx)          # mx = f * 2**e, f in [0.5, 1)
                scales[bi, bj] = math.ldexp(1.0, e - 1 if f == 0.5 else e)
    s_full = np.repeat(np.repeat(scales, block, 0), block, 1)[:m, :n]
    bits = philox.round_bf16_bits(A / s_full)
    return bits, scales.astype(np.float32)


def block_dequantize_bf16(bits: np.ndarray, scales: np.ndarray, block: int = 128):
    m, n = bits.shape
    s_full = np.repeat(np.repeat(scales.astype(np.float64), block, 0), block, 1)[:m, :n]
    return philox.bf16_bits_to_f64(bits) * s_full


# ----------------------------------------------------------------------------- GN steps
def sketch_pass(A: np.ndarray, X: np.ndarray, Y: np.ndarray):
    """AX and Y^T A (Algorithm 2.1 step 2)."""
    return A @ X, Y.T @ A


@dataclass
class Core:
    C: np.ndarray        # (r+l) x r core Y^T (AX)
    Q: np.ndarray        # (r+l) x r, Householder Q with R_ii >= 0
    R: np.ndarray        # r x r upper triangular
    k: int               # numerical rank kept (prefix rule)
    Q2: np.ndarray       # r x k (identity columns when k == r)
    R2: np.ndarray       # k x k upper triangular (R itself when k == r)
    tau: float
    non_monotone: bool   # some |R_jj| >= tau after the first one below tau
    status: int          # 0 ok, 7 numeric (non-finite diagonal or k == 0)


def _qr_nonneg(M: np.ndarray):
    """Economic Householder QR (LAPACK geqrf/orgqr) with a non-negative R diagonal."""
    Q, R = sla.qr(M, mode="economic")
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * s[None, :], R * s[:, None]


def core(AX: np.ndarray, Y: np.ndarray, tau: float) -> Core:
    """Core matrix, its QR and the epsilon-truncation (Alg. 2.1 step 2; Sec. 5.1.1)."""
    return core_of(Y.T @ AX, tau)


def core_right(YA: np.ndarray, X: np.ndarray, tau: float) -> Core:
    """The same with the core matrix formed as (Y^T A) X, the order the cost
    count of Section 2.3 uses (a fast transform of the rows of Y^T A when X is
    structured)."""
    return core_of(YA @ X, tau)


def core_of(C: np.ndarray, tau: float) -> Core:
    """QR of a given core matrix C ((r+l) x r) and the epsilon-truncation."""
    r = C.shape[1]
    Q, R = _qr_nonneg(C)
    d = np.abs(np.diag(R))
    # keep |R_ii| >= tau; with tau <= 0 (plain GN) keep every non-zero diagonal.
    # NaN fails both comparisons.
    bad = ~(d >= tau) if tau > 0 else ~(d > 0)
    k = int(np.argmax(bad)) if bad.any() else r
    non_monotone = bool(np.any(~bad[k:])) if k < r else False
    status = 0
    if not np.all(np.isfinite(np.diag(R))) or k == 0:
        status = 7
    if k == r:
        Q2, R2 = np.eye(r), R.copy()
    elif k == 0:
        Q2, R2 = np.zeros((r, 0)), np.zeros((0, 0))
    else:
        Q2, R2 = _qr_nonneg(R[:k, :].T)     # R_1^T = Q_2 R_2
    return Core(C=C, Q=Q, R=R, k=k, Q2=Q2, R2=R2, tau=tau,
                non_monotone=non_monotone, status=status)


def factors(AX: np.ndarray, YA: np.ndarray, c: Core):
    """F (m x k) and G (k x n) with A_hat = F G.

    k == r : F = (AX) R^-1 by a triangular solve, G = Q^T (Y^T A)  (Sec. 5.1)
    k <  r : F = (AX Q_2) R_2^{-T},           G = Q_1^T (Y^T A)   (Sec. 5.1.1)
    """
    k, r = c.k, c.R.shape[0]
    if k == r:
        F = sla.solve_triangular(c.R, AX.T, trans="T", lower=False).T
    else:
        F = sla.solve_triangular(c.R2, (AX @ c.Q2).T, trans="N", lower=False).T
    G = c.Q[:, :k].T @ YA
    return F, G


def apply_right(AX, YA, c: Core, W):
    """A_hat W evaluated as AX (R^-1 (Q^T (Y^T A W)))  (Section 2)."""
    k, r = c.k, c.R.shape[0]
    t = c.Q[:, :k].T @ (YA @ W)
    if k == r:
        t = sla.solve_triangular(c.R, t, lower=False)
    else:
        t = c.Q2 @ sla.solve_triangular(c.R2, t, trans="T", lower=False)
    return AX @ t


def apply_left(AX, YA, c: Core, W):
    """W A_hat evaluated as (((W AX) R^-1) Q^T) Y^T A  (Section 2)."""
    k, r = c.k, c.R.shape[0]
    t = W @ AX
    if k == r:
        t = sla.solve_triangular(c.R, t.T, trans="T", lower=False).T
    else:
        t = sla.solve_triangular(c.R2, (t @ c.Q2).T, trans="N", lower=False).T
    return (t @ c.Q[:, :k].T) @ YA


def residual_fro(A: np.ndarray, F: np.ndarray, G: np.ndarray, rows: int = 1024) -> float:
    """||A - F G||_F formed block row by block row (no Gram-matrix shortcut)."""
    acc = 0.0
    for i0 in range(0, A.shape[0], rows):
        D = A[i0:i0 + rows] - F[i0:i0 + rows] @ G
        acc += float(np.sum(D * D))
    return math.sqrt(acc)


def diff_fro(F1, G1, F2, G2, rows: int = 1024) -> float:
    """||F1 G1 - F2 G2||_F, block row by block row."""
    acc = 0.0
    for i0 in range(0, F1.shape[0], rows):
        D = F1[i0:i0 + rows] @ G1 - F2[i0:i0 + rows] @ G2
        acc += float(np.sum(D * D))
    return math.sqrt(acc)


@dataclass
class GNResult:
    AX: np.ndarray
    YA: np.ndarray
    core: Core
    F: np.ndarray
    G: np.ndarray

    @property
    def approx(self) -> np.ndarray:
        return self.F @ self.G


def gn(A, X, Y, tau: float) -> GNResult:
    """The whole (S)GN pipeline with explicit sketches (Algorithm 2.1 + Sec. 5.1.1)."""
    AX, YA = sketch_pass(A, X, Y)
    c = core(AX, Y, tau)
    F, G = factors(AX, YA, c)
    return GNResult(AX=AX, YA=YA, core=c, F=F, G=G)


# ----------------------------------------------------------------------------- comparison formulas (pins)
def pinv_eps_svd(C: np.ndarray, eps: float) -> np.ndarray:
    """(C)_eps^+ = V_1 Sigma_1^-1 U_1^T over singular values > eps (Section 2)."""
    U, s, Vt = np.linalg.svd(C, full_matrices=False)
    keep = s > eps
    return (Vt[keep].T / s[keep]) @ U[:, keep].T


def gn_svd(A, X, Y, eps: float) -> np.ndarray:
    """SGN with the SVD-based epsilon-pseudoinverse (Section 5.1.1, first option)."""
    AX, YA = A @ X, Y.T @ A
    return (AX @ pinv_eps_svd(Y.T @ AX, eps)) @ YA


def hmt(A, Omega) -> np.ndarray:
    """HMT range finder Q (Q^T A), Q = orth(A Omega) (Algorithm 1.1)."""
    Q, _ = np.linalg.qr(A @ Omega)
    return Q @ (Q.T @ A)


def tropp17(A, X, Y) -> np.ndarray:
    """Q (Y^T Q)^+ Y^T A with AX = QR (Section 2.4); equal to plain GN in exact
    arithmetic."""
    Q, _ = np.linalg.qr(A @ X)
    B = np.linalg.lstsq(Y.T @ Q, Y.T @ A, rcond=None)[0]
    return Q @ B


def nystrom_psd(A, X) -> np.ndarray:
    """Classical Nystrom AX (X^T A X)^-1 (AX)^T for A positive definite (eq. (1))."""
    AX = A @ X
    cf = sla.cho_factor(X.T @ AX)
    return AX @ sla.cho_solve(cf, AX.T)


def cur(A, rows, cols) -> np.ndarray:
    """A[:, J] (A[I, J])^+ A[I, :] -- GN with identity-column sketches (Sec. 2.4.1)."""
    B = np.linalg.lstsq(A[np.ix_(rows, cols)], A[rows, :], rcond=None)[0]
    return A[:, cols] @ B


# ----------------------------------------------------------------------------- theory
def optimal_error(sigma: np.ndarray, r: int) -> float:
    """||A - A_r||_F = sqrt(sum_{i>r} sigma_i^2) for a known spectrum."""
    s = np.asarray(sigma, np.float64)
    return float(np.sqrt(np.sum(s[r:] ** 2)))


def hmt_bound(sigma, r: int) -> float:
    """min over rhat <= r-2 of sqrt(1 + r/(r-rhat-1)) ||A - A_rhat||_F (Thm 3.1)."""
    return min(math.sqrt(1 + r / (r - rh - 1)) * optimal_error(sigma, rh)
               for rh in range(0, r - 1))


def gn_bound(sigma, r: int, l: int) -> float:
    """Theorem 3.2: sqrt(1 + (r+l)/(l-1)) times the Theorem 3.1 bound (l >= 2)."""
    return math.sqrt(1 + (r + l) / (l - 1)) * hmt_bound(sigma, r)


def gn_over_hmt_factor(r: int, l: int) -> float:
    """sqrt(1 + (r+l)/(l-1)): E||E_GN||_F over sqrt(E||E_HMT||_F^2) (Thm 3.2)."""
    return math.sqrt(1 + (r + l) / (l - 1))
