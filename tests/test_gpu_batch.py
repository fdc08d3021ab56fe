"""Batched solves (gn_batch_prepare / gn_batch_solve) against the FP64 oracle and
the single-problem path -- needs a GPU.

A batch of the batched workload's recipe (sigma_i = 10^(-8 i / n), Gaussian X and
Y, r + l <= 192): ten problems at reduced sizes, r close to n, a tiny r, and two at
the workload's largest sizes (4096 x 3000 with r = 128; 4000 x 700 with r = 100):
  * every problem's AX and Y^T A against FP64 products of the same FP32 inputs,
    entrywise within gamma_K of the magnitudes (FP32 accumulation over K terms);
  * every problem's kept rank against the oracle, and its error ||A - A_hat||_F
    within 1.05x the FP64 oracle's (same sketch values), or, where the oracle's
    error is below what FP32 resolves (100 u32 ||A||_F), within that floor;
  * replaying a captured HIP graph of the solve reproduces the eager results bit
    for bit, with eager work between replays;
  * every tile policy gives the same kept ranks and passes the same checks.
"""
import math
import os
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import gn as OG  # noqa: E402
from paper_2009_11392_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_11392_amd import gn
    return gn


def host(t):
    return t.detach().cpu().double().numpy()


def gamma(K):
    return K * U32 / (1 - K * U32)


@pytest.fixture(scope="module")
def batch_inputs(G):
    specs = W.batch_specs(10, seed=4, m_range=(256, 900), r_range=(8, 128))
    specs.append(W.BatchSpec(200, 130, 128, 64, (4 << 32) + 99, 40099))   # r close to n
    specs.append(W.BatchSpec(300, 140, 9, 5, (4 << 32) + 98, 40098))      # small r
    specs.append(W.BatchSpec(4096, 3000, 128, 64, (4 << 32) + 97, 40097))  # the largest sizes
    specs.append(W.BatchSpec(4000, 700, 100, 50, (4 << 32) + 96, 40096))   # tall, long K
    mats = [W.batch_host_matrix(b) for b in specs]
    probs = []
    for b, A in zip(specs, mats):
        p = G.Problem(b.m, b.n, b.r, b.l, seed=b.seed, mode="f32", eps=10 * U32)
        ld = (b.n + 3) // 4 * 4
        Ad = torch.zeros(b.m, ld, dtype=torch.float32, device="cuda")
        Ad[:, :b.n] = torch.from_numpy(A).float().cuda()
        probs.append((p, Ad[:, :b.n]))
    return specs, mats, probs


def _check(G, specs, mats, batch):
    for i, (b, A) in enumerate(zip(specs, mats)):
        p = batch.problems[i]
        A32 = A.astype(np.float32).astype(np.float64)
        X, Y = OG.gaussian_sketches(b.seed, b.m, b.n, b.r, b.l, mode="f32")
        AX = host(batch.AX[i])
        YtA = host(batch.YtA[i])
        assert np.all(np.abs(AX - A32 @ X) <= gamma(b.n) * (np.abs(A32) @ np.abs(X)) + 1e-30), i
        assert np.all(np.abs(YtA - Y.T @ A32) <= gamma(b.m) * (np.abs(Y.T) @ np.abs(A32)) + 1e-30), i
        tau = OG.threshold(p.eps, OG.nu_gaussian(b.n, b.r), OG.nu_gaussian(b.m, b.r + b.l))
        ref = OG.gn(A, X, Y, tau)
        core = batch.core[i]
        assert core.rank() == ref.core.k, (i, core.rank(), ref.core.k)
        assert (core.flags() & 3) == 0
        F, Gm = G.gn_factors(p, batch.AX[i], batch.YtA[i], core)
        Ad = torch.from_numpy(A).cuda()
        e = math.sqrt(float(G.gn_residual(Ad, F, Gm).item()))
        e_ref = OG.residual_fro(A, ref.F, ref.G)
        floor = 100 * U32 * np.linalg.norm(A)
        if e_ref >= floor:
            assert e <= 1.05 * e_ref, (i, e, e_ref)
        else:
            assert e <= floor, (i, e, floor)


def test_batch_matches_oracle(G, batch_inputs):
    specs, mats, probs = batch_inputs
    batch = G.Batch(probs)
    assert batch.plan.count == len(probs)
    batch.solve()
    torch.cuda.synchronize()
    _check(G, specs, mats, batch)


@pytest.mark.parametrize("policy", [(1, 1, 1, 1), (0, 0, 2, 2), (2, 1, 0, 1), (3, 3, 4, 4),
                                    (4, 4, 3, 3)])
def test_batch_tile_policies(G, batch_inputs, policy):
    specs, mats, probs = batch_inputs
    batch = G.Batch(probs, tile_policy=policy)
    assert tuple(batch.plan.tile_policy) == policy
    batch.solve()
    torch.cuda.synchronize()
    _check(G, specs, mats, batch)


def test_batch_graph_replay(G, batch_inputs):
    specs, mats, probs = batch_inputs
    batch = G.Batch(probs)
    batch.solve()
    torch.cuda.synchronize()
    ref = [(ax.clone(), yta.clone(), c.R.clone(), c.Q1.clone(), c.k.clone())
           for ax, yta, c in zip(batch.AX, batch.YtA, batch.core)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.solve()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.solve()
    for rep in range(3):
        for ax, yta in zip(batch.AX, batch.YtA):   # clobber outputs between replays
            ax.fill_(float("nan"))
            yta.zero_()
        junk = torch.randn(1024, 1024, device="cuda") @ torch.randn(1024, 1024, device="cuda")
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        del junk
        for (ax0, yta0, r0, q0, k0), ax, yta, c in zip(ref, batch.AX, batch.YtA, batch.core):
            assert torch.equal(ax, ax0) and torch.equal(yta, yta0), rep
            assert torch.equal(c.R, r0) and torch.equal(c.Q1, q0) and torch.equal(c.k, k0), rep
