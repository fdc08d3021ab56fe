"""Seeded synthetic inputs for the GN sketch library (test matrices, loss weights).

This module generates *inputs* only: matrices with a controlled spectrum, built
as A = U diag(sigma) V^T (+ entrywise Gaussian noise) with U and V the Q factors
of seeded Gaussian matrices -- the construction of the paper's experiments
(Section 2.1 and Section 7.1, "U, V obtained via the QR factorization of
Gaussian matrices").  It holds none of GN's arithmetic and uses its own random
streams (NumPy PCG64 on the host, torch's generator on the device), so it is
independent of both the HIP sketch generators and the CPU oracle; both of those
consume what it produces.

The workloads (sizes, spectra, sketch kinds, precisions) are the ones the
library is measured on:

  small    : 2000 x 1000 FP64, sigma_i = 0.9^i, Gaussian X, Y, r = 50, l = 25,
             eps = 1e-15 ||A||_2.  The CPU oracle finishes it in seconds.
  srht32k  : 32768 x 32768 FP32, sigma_i = i^-2 (i <= 4096) plus 1e-6 i.i.d.
             Gaussian noise; SRHT X with r = 1000, Gaussian Y with r + l = 1500.
  bf16_32k : the same matrix stored as bfloat16 with one power-of-two FP32 scale
             per 128 x 128 block; Gaussian X, Y (r = 2000, l = 1000).
  f16_32k  : the same, stored as IEEE binary16 with the same block scales.
  grad8k   : 8192 x 4096 FP32, sigma_i = i^-1.5, Gaussian X, Y (r = 256, l = 128).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

U_F32 = 2.0 ** -24
U_F64 = 2.0 ** -53


@dataclass(frozen=True)
class Workload:
    name: str
    m: int
    n: int
    r: int
    l: int
    kind_x: str             # "gaussian" | "srht"
    kind_y: str             # "gaussian"
    mode: str               # "f64" | "f32" | "bf16"
    seed: int               # sketch seed (X, Y, SRHT)
    spectrum: str           # "geometric0.9" | "poly2" | "poly1.5"
    rank: int               # number of nonzero signal singular values
    noise: float            # entrywise noise standard deviation
    eps_rel: float          # eps / sigma_1
    input_seed: int = 1000  # seed of the input generator (A, G)

    def sigma(self) -> np.ndarray:
        i = np.arange(1, self.rank + 1, dtype=np.float64)
        if self.spectrum == "geometric0.9":
            return 0.9 ** i
        if self.spectrum == "poly2":
            return i ** -2.0
        if self.spectrum == "poly1.5":
            return i ** -1.5
        raise ValueError(self.spectrum)

    @property
    def eps(self) -> float:
        return self.eps_rel * float(self.sigma()[0])

    def scaled(self, m: int, n: int, r: int | None = None, l: int | None = None,
               rank: int | None = None, name: str | None = None) -> "Workload":
        """Same recipe at another size (for parity tests that span several tiles)."""
        r = self.r if r is None else r
        l = (r + 1) // 2 if l is None else l
        rank = min(m, n, self.rank if rank is None else rank)
        return Workload(name or f"{self.name}@{m}x{n}r{r}", m, n, r, l, self.kind_x,
                        self.kind_y, self.mode, self.seed, self.spectrum, rank,
                        self.noise, self.eps_rel, self.input_seed)


SMALL = Workload("small_2000x1000_f64", 2000, 1000, 50, 25, "gaussian", "gaussian",
                 "f64", seed=1, spectrum="geometric0.9", rank=1000, noise=0.0,
                 eps_rel=1e-15)
SRHT32K = Workload("srht_32768x32768_f32", 32768, 32768, 1000, 500, "srht", "gaussian",
                   "f32", seed=2, spectrum="poly2", rank=4096, noise=1e-6,
                   eps_rel=10 * U_F32)
# small r: the pass moves 4 bytes of A per 2(r+l) + log2 n' = 45 flops, below the
# FP32 ridge (19.7 flop/B), so it is bound by HBM bandwidth, not the matrix cores
SRHT32K_R10 = Workload("srht_32768x32768_f32_r10", 32768, 32768, 10, 5, "srht", "gaussian",
                       "f32", seed=2, spectrum="poly2", rank=4096, noise=1e-6,
                       eps_rel=10 * U_F32)
BF16_32K = Workload("bf16bs_32768x32768", 32768, 32768, 2000, 1000, "gaussian",
                    "gaussian", "bf16", seed=3, spectrum="poly2", rank=4096, noise=1e-6,
                    eps_rel=10 * U_F32)
F16_32K = Workload("f16bs_32768x32768", 32768, 32768, 2000, 1000, "gaussian",
                   "gaussian", "f16", seed=3, spectrum="poly2", rank=4096, noise=1e-6,
                   eps_rel=10 * U_F32)
F32_32K = Workload("f32_32768x32768_gauss", 32768, 32768, 2000, 1000, "gaussian",
                   "gaussian", "f32", seed=3, spectrum="poly2", rank=4096, noise=1e-6,
                   eps_rel=10 * U_F32)
GRAD8K = Workload("grad_8192x4096_f32", 8192, 4096, 256, 128, "gaussian", "gaussian",
                  "f32", seed=5, spectrum="poly1.5", rank=4096, noise=0.0,
                  eps_rel=10 * U_F32)

ALL = {w.name: w for w in (SMALL, SRHT32K, SRHT32K_R10, BF16_32K, F16_32K, F32_32K, GRAD8K)}


@dataclass(frozen=True)
class BatchSpec:
    """One problem of the batched workload: sizes, sketch seed, input seed."""
    m: int
    n: int
    r: int
    l: int
    seed: int
    input_seed: int

    def sigma(self) -> np.ndarray:
        """sigma_i = 10^(-8 i / n), i = 1 .. n."""
        i = np.arange(1, self.n + 1, dtype=np.float64)
        return 10.0 ** (-8.0 * i / self.n)


def batch_specs(count: int = 512, seed: int = 4, m_range=(256, 4096), r_range=(8, 128)):
    """The batched workload: m ~ U[m_range], n ~ U[128, m], r ~ U[r_range] (integers,
    inclusive), l = ceil(r/2); sketch seed of problem p = (seed << 32) + p."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(count):
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(128, m + 1))
        r = int(rng.integers(r_range[0], r_range[1] + 1))
        out.append(BatchSpec(m, n, r, (r + 1) // 2, (seed << 32) + p, 40000 + p))
    return out


def batch_host_matrix(b: BatchSpec) -> np.ndarray:
    return spectrum_matrix(b.m, b.n, b.sigma(), b.input_seed)


def batch_device_matrix(b: BatchSpec, device="cuda", host_factors: bool = False):
    """A of problem b built on the device in FP32 (torch generator seeded with the
    input seed; U, V Q factors of Gaussians), row stride a multiple of 4.  With
    `host_factors` the matrix is built on the host (`batch_host_matrix`) and copied
    over, so that no library kernel runs on the device."""
    import torch
    ld = (b.n + 3) // 4 * 4
    A = torch.zeros(b.m, ld, dtype=torch.float32, device=device)
    if host_factors:
        A[:, :b.n] = torch.from_numpy(batch_host_matrix(b).astype(np.float32)).to(device)
        return A[:, :b.n]
    g = torch.Generator(device=device)
    g.manual_seed(b.input_seed)
    k = b.n
    sig = torch.tensor(b.sigma(), dtype=torch.float64, device=device)
    U, _ = torch.linalg.qr(torch.randn(b.m, k, generator=g, device=device, dtype=torch.float64))
    V, _ = torch.linalg.qr(torch.randn(b.n, k, generator=g, device=device, dtype=torch.float64))
    A[:, :b.n] = ((U * sig[None, :]) @ V.T).to(torch.float32)
    return A[:, :b.n]


# ----------------------------------------------------------------------------- host (NumPy)
def _orth_host(rng: np.random.Generator, rows: int, k: int) -> np.ndarray:
    q, _ = np.linalg.qr(rng.standard_normal((rows, k)))
    return q


def spectrum_matrix(m: int, n: int, sigma: np.ndarray, seed: int,
                    noise: float = 0.0) -> np.ndarray:
    """FP64 A = U diag(sigma) V^T + noise * N on the host (PCG64 seeded by `seed`)."""
    rng = np.random.default_rng(seed)
    k = len(sigma)
    U = _orth_host(rng, m, k)
    V = _orth_host(rng, n, k)
    A = (U * np.asarray(sigma)[None, :]) @ V.T
    if noise:
        A += noise * rng.standard_normal((m, n))
    return A


def host_matrix(w: Workload) -> np.ndarray:
    return spectrum_matrix(w.m, w.n, w.sigma(), w.input_seed, w.noise)


def integer_matrix(rows: int, cols: int, seed: int, lo: int = -3, hi: int = 3) -> np.ndarray:
    """Small-integer matrix (for exact rational checks)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(rows, cols)).astype(np.float64)


def host_gaussian(rows: int, cols: int, seed: int) -> np.ndarray:
    """Seeded FP64 Gaussian input (loss weights, right-hand sides W)."""
    return np.random.default_rng(seed).standard_normal((rows, cols))


# ----------------------------------------------------------------------------- device (torch)
def device_matrix(w: Workload, device="cuda", dtype=None, host_factors: bool = False):
    """A of workload `w` built on the device in FP32 (or `dtype`), seeded.

    U and V are the Q factors of Gaussian (m x k) and (n x k) matrices drawn with
    torch's device generator; A = (U * sigma) V^T, then entrywise noise is added
    block by block to bound temporary memory.

    With `host_factors` the orthonormal factors and their FP32 product are made
    on the host instead (NumPy PCG64 and LAPACK; the same recipe with other
    random numbers) and only the noise is drawn on the device.  That route runs
    no library kernel on the device (no QR, no GEMM), which is what hardware
    counter collection needs; it takes tens of seconds of host time at 32768^2.
    """
    import torch
    dtype = dtype or torch.float32
    g = torch.Generator(device=device)
    g.manual_seed(w.input_seed)
    k = w.rank
    if host_factors:
        rng = np.random.default_rng(w.input_seed)
        Us = (_orth_host(rng, w.m, k) * w.sigma()[None, :]).astype(np.float32)
        Vt = np.ascontiguousarray(_orth_host(rng, w.n, k).T.astype(np.float32))
        A = torch.from_numpy(Us @ Vt).to(device)
        del Us, Vt
    else:
        sig = torch.tensor(w.sigma(), dtype=torch.float64, device=device)

        def orth(rows):
            G = torch.randn(rows, k, generator=g, device=device, dtype=torch.float64)
            q, _ = torch.linalg.qr(G)
            return q

        U = orth(w.m)
        V = orth(w.n)
        A = ((U * sig[None, :]).to(torch.float32) @ V.to(torch.float32).T)
        del U, V
    if w.noise:
        step = max(1, (1 << 26) // w.n)
        for i0 in range(0, w.m, step):
            i1 = min(w.m, i0 + step)
            A[i0:i1].add_(torch.randn(i1 - i0, w.n, generator=g, device=device,
                                      dtype=torch.float32), alpha=w.noise)
    return A.to(dtype)


def device_gaussian(rows: int, cols: int, seed: int, device="cuda", dtype=None):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.randn(rows, cols, generator=g, device=device,
                       dtype=dtype or torch.float32)
