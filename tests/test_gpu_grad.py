"""GPU reverse mode (gn_backward, GNApprox) against the FP64 oracle -- needs a GPU.

FP64 mode is compared element by element (relative Frobenius) with
oracle.grad.gn_backward on the same seeded inputs: 1e-10 for k = r, 1e-9 for a
truncated core.  FP32 mode is compared with the FP64 oracle run on the FP32
values of A, X and Y, within a tolerance derived from the arithmetic: the FP32
pass products (length-K sums, K = max(m, n)) carry relative errors of order
sqrt(K) u32, which the core adjoint amplifies by at most the condition number
kappa of the kept core; the test allows 10 kappa sqrt(K) u32.
"""
import math
import os
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import gn as OG, grad as OGR  # noqa: E402
from paper_2009_11392_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_11392_amd import gn
    return gn


def dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def host(t):
    return t.detach().cpu().double().numpy()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _tau(p):
    if p.eps <= 0:
        return 0.0
    return OG.threshold(p.eps, OG.nu_gaussian(p.n, p.r), OG.nu_gaussian(p.m, p.rl))


def _case(G, m, n, r, l, sig, seed, eps=0.0, mode="f64"):
    A = W.spectrum_matrix(m, n, np.asarray(sig), seed=seed)
    Gb = W.host_gaussian(m, n, seed + 1)
    p = G.Problem(m, n, r, l, seed=seed + 2, mode=mode, eps=eps)
    return A, Gb, p


@pytest.mark.parametrize("m,n,r,l", [(300, 200, 20, 10), (517, 389, 33, 17)])
def test_backward_f64_matches_oracle(G, m, n, r, l):
    sig = np.arange(1, min(m, n) + 1, dtype=float) ** -1.5
    A, Gb, p = _case(G, m, n, r, l, sig, seed=m)
    X, Y = OG.gaussian_sketches(p.seed, m, n, r, l)
    ref_core = OG.gn(A, X, Y, _tau(p)).core
    assert ref_core.k == r
    ref = OGR.gn_backward(A, X, Y, ref_core, Gb)
    Ad = dev(A)
    AX, YtA, core = G.solve(p, Ad)
    assert core.rank() == r
    dA = G.gn_backward(p, dev(Gb), YtA, core, AX=AX)
    assert relerr(host(dA), ref) <= 1e-10
    # AX recomputed from A inside gn_backward: the same FP64 criterion against the
    # oracle; against the first result it differs only in the order of the AX sums
    # (the pass splits K, the recomputation reads X transposed)
    dA2 = G.gn_backward(p, dev(Gb), YtA, core, A=Ad)
    assert relerr(host(dA2), ref) <= 1e-10
    assert relerr(host(dA2), host(dA)) <= 1e-11
    # AX passed with a row stride larger than r
    AXw = torch.zeros(m, r + 5, dtype=torch.float64, device="cuda")
    AXw[:, :r] = AX
    dA3 = G.gn_backward(p, dev(Gb), YtA, core, AX=AXw[:, :r])
    assert torch.equal(dA3, dA)


def test_backward_f64_truncated_core(G):
    m, n, r, l = 300, 200, 20, 10
    sig = np.r_[np.linspace(1.0, 0.2, 14), 1e-9 * np.ones(186)]
    A, Gb, p = _case(G, m, n, r, l, sig, seed=41, eps=1e-6)
    X, Y = OG.gaussian_sketches(p.seed, m, n, r, l)
    ref_core = OG.gn(A, X, Y, _tau(p)).core
    assert ref_core.k == 14
    ref = OGR.gn_backward(A, X, Y, ref_core, Gb)
    AX, YtA, core = G.solve(p, dev(A))
    assert core.rank() == 14
    dA = G.gn_backward(p, dev(Gb), YtA, core, AX=AX)
    assert relerr(host(dA), ref) <= 1e-9


# gn_backward forks the core-only part of the adjoint, and later U's first term
# and V, onto the per-device side stream and joins it back twice.  Two backward
# calls enqueued at once on two streams (one with a truncated core), each with its
# own workspace, give bit for bit the results of the same calls one at a time.
def test_backward_on_two_streams(G):
    m, n, r, l = 300, 200, 20, 10
    cases = [_case(G, m, n, r, l, np.arange(1, 201, dtype=float) ** -1.5, seed=300),
             _case(G, m, n, r, l, np.r_[np.linspace(1.0, 0.2, 14), 1e-9 * np.ones(186)], seed=41,
                   eps=1e-6)]
    solved = []
    for A, Gb, p in cases:
        AX, YtA, core = G.solve(p, dev(A))
        solved.append((p, dev(Gb), AX, YtA, core))
    torch.cuda.synchronize()
    assert [c[4].rank() for c in solved] == [r, 14]
    serial = [G.gn_backward(p, Gbd, YtA, core, AX=AX) for p, Gbd, AX, YtA, core in solved]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    both = []
    for (p, Gbd, AX, YtA, core), st in zip(solved, streams):
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            both.append(G.gn_backward(p, Gbd, YtA, core, AX=AX))
    torch.cuda.synchronize()
    for a, b in zip(serial, both):
        assert torch.equal(a, b)


def test_autograd_function_f64(G):
    m, n, r, l = 256, 160, 16, 8
    sig = np.arange(1, 161, dtype=float) ** -1.5
    A, Gb, p = _case(G, m, n, r, l, sig, seed=7)
    X, Y = OG.gaussian_sketches(p.seed, m, n, r, l)
    res = OG.gn(A, X, Y, _tau(p))
    for store_ax in (True, False):
        Ad = dev(A).requires_grad_(True)
        Ahat = G.gn_approx(Ad, p, store_ax)
        assert relerr(host(Ahat), res.approx) <= 1e-10
        (dev(Gb) * Ahat).sum().backward()
        assert relerr(host(Ad.grad), OGR.gn_backward(A, X, Y, res.core, Gb)) <= 1e-10


def test_finite_differences_on_gpu_f64(G):
    """64 x 32, r = 4: <dA, E> against central differences of the GPU forward."""
    m, n, r, l = 64, 32, 4, 2
    sig = np.linspace(1.0, 0.3, 32)
    A, Gb, p = _case(G, m, n, r, l, sig, seed=3)
    Gd = dev(Gb)
    Ad = dev(A).requires_grad_(True)
    (Gd * G.gn_approx(Ad, p)).sum().backward()
    dA = Ad.grad
    rng = np.random.default_rng(9)
    h = 1e-6
    for _ in range(3):
        E = dev(rng.standard_normal((m, n)))
        with torch.no_grad():
            lp = float((Gd * G.gn_approx(dev(A) + h * E, p)).sum())
            lm = float((Gd * G.gn_approx(dev(A) - h * E, p)).sum())
        fd = (lp - lm) / (2 * h)
        an = float((dA * E).sum())
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-3 * float(dA.norm()))


def test_backward_f32_within_conditioning_bound(G):
    """The gradient workload's recipe (sigma_i = i^-1.5, Gaussian X and Y) at
    1024 x 512, r = 64, l = 32, FP32 mode."""
    m, n, r, l = 1024, 512, 64, 32
    sig = np.arange(1, 513, dtype=float) ** -1.5
    A, Gb, p = _case(G, m, n, r, l, sig, seed=5, eps=10 * U32, mode="f32")
    A32 = A.astype(np.float32).astype(np.float64)
    G32 = Gb.astype(np.float32).astype(np.float64)
    X, Y = OG.gaussian_sketches(p.seed, m, n, r, l, mode="f32")
    ref_core = OG.gn(A32, X, Y, _tau(p)).core
    assert ref_core.k == r
    ref = OGR.gn_backward(A32, X, Y, ref_core, G32)
    AX, YtA, core = G.solve(p, dev(A, torch.float32))
    assert core.rank() == r
    dA = G.gn_backward(p, dev(Gb, torch.float32), YtA, core, AX=AX)
    assert dA.dtype == torch.float32
    d = np.abs(np.diag(ref_core.R))
    kappa = float(d.max() / d.min())
    tol = 10 * kappa * math.sqrt(max(m, n)) * U32
    err = relerr(host(dA), ref)
    assert err <= tol, (err, tol)
    # recomputed AX agrees with the stored one to FP32 roundoff
    dA2 = G.gn_backward(p, dev(Gb, torch.float32), YtA, core, A=dev(A, torch.float32))
    assert relerr(host(dA2), host(dA)) <= tol


def test_materialize_matches_factors(G):
    m, n, r, l = 300, 200, 20, 10
    sig = np.arange(1, 201, dtype=float) ** -1.5
    A, _, p = _case(G, m, n, r, l, sig, seed=13)
    AX, YtA, core = G.solve(p, dev(A))
    F, Gm = G.gn_factors(p, AX, YtA, core)
    Ahat = G.gn_materialize(p, AX, YtA, core)
    assert relerr(host(Ahat), host(F) @ host(Gm)) <= 1e-13
