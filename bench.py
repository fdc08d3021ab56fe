"""Benchmark of the GN hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-compare] [--no-cpu] [--no-error]

One step = one generalized Nystrom solve of the workload's matrix: the sketches
(Philox Gaussian Y, SRHT signs and sample or Gaussian X), the single fused pass
over A (AX and Y^T A), the core (C = Y^T (AX), Householder QR, eps-truncation,
second QR when truncated) and one product with the factors (A_hat W, 16
columns).  The inputs are resident in HBM before timing starts.  HIP events on
the library's stream (torch's current stream) time each stage; `value` is the
pass's algorithmic TFLOP/s.  After timing: the error ||A - A_hat||_F (tile-wise
on the device), a bounded CPU-oracle baseline, and the BF16-vs-FP32 comparison
on the 32768^2, r = 2000, l = 1000 shape (same matrix), the reverse mode on the
8192 x 4096 gradient workload (forward, backward, backward with AX recomputed),
the 512-problem batched workload (pass launch, whole solve, graph replay),
and the core under each Section 5.1.1 stabilization with the Section 5.1.2 check.
Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": 157.3, "bf16": 2500.0, "f16": 2500.0, "f64": 78.6}   # dense TFLOP/s (MI355X datasheet)
HBM_PEAK_GBS = 8000.0
METRIC = "sketch-pass GB/s & TFLOP/s; GN solves/sec bf16 vs fp32 at equal error"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def srht_pad(n):
    """Hadamard order n' = smallest power of two >= n (Section 3.1)."""
    return 1 << max(0, int(n - 1).bit_length())


def pass_algorithmic(w, npad):
    """(flops, bytes) the pass must do / move: A once, sketches once, outputs once."""
    m, n, r, rl = w.m, w.n, w.r, w.r + w.l
    es = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[w.mode]
    acc = 8 if w.mode == "f64" else 4
    flops = 2.0 * m * n * rl
    byts = m * n * es + m * rl * es + (m * r + rl * n) * acc
    if w.kind_x == "srht":
        flops += m * n * math.log2(npad)
        byts += npad + 4 * r
    else:
        flops += 2.0 * m * n * r
        byts += n * r * es
    if w.mode in ("bf16", "f16"):
        byts += 4 * ((m + 127) // 128) * ((n + 127) // 128)
    return flops, byts


def source_hash():
    h = hashlib.sha256()
    for f in ("pass.hip", "pass_narrow.hip", "gemm_tiles.h", "gemm_h16.h", "gn_internal.h",
              "lane_ops.h"):
        with open(os.path.join(ROOT, "paper_2009_11392_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload):
    path = os.path.join(ROOT, "profiles", "pass_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    ent = rec.get(workload)
    if not ent or ent.get("sources_sha") != source_hash():
        return None
    return ent.get("hbm_bytes_per_launch")


def optimum_estimate(w):
    """||A - A_r||_F for sigma plus i.i.d. noise: sqrt(sum_{i>r} sigma_i^2 +
    nu^2 (m-r)(n-r)) -- an estimate (the noise spectrum is not closed-form)."""
    s = w.sigma()
    return math.sqrt(float((s[w.r:] ** 2).sum()) + w.noise ** 2 * (w.m - w.r) * (w.n - w.r))


class Runner:
    """Preallocated buffers and one timed solve for a workload."""

    def __init__(self, gn, w, A, scales=None, kc=16, A_ref=None):
        import torch
        self.gn, self.w, self.A, self.scales = gn, w, A, scales
        # the matrix the error is measured against: the unquantized FP32 matrix for
        # the block-scaled BF16 variant, A itself otherwise
        self.A_ref = A if A_ref is None else A_ref
        self.p = gn.Problem(w.m, w.n, w.r, w.l, kind_x=w.kind_x, kind_y=w.kind_y, seed=w.seed,
                            mode=w.mode, eps=w.eps)
        acc = gn.ACCUM_TORCH[w.mode]
        self.ws = gn.workspace(self.p, gn.C.GN_OP_SKETCH)
        self.ws_core = gn.workspace(self.p, gn.C.GN_OP_CORE)
        self.AX = torch.empty(w.m, w.r, dtype=acc, device="cuda")
        self.YtA = torch.empty(self.p.rl, w.n, dtype=acc, device="cuda")
        self.core = gn.new_core(self.p)
        g = torch.Generator(device="cuda")
        g.manual_seed(99)
        self.W = torch.randn(w.n, kc, generator=g, device="cuda", dtype=torch.float64)
        self.out = torch.empty(w.m, kc, dtype=torch.float64, device="cuda")

    def step(self, ev):
        gn, p = self.gn, self.p
        ev[0].record()
        gn.gn_sketch_prepare(p, self.ws)
        ev[1].record()
        gn.gn_sketch_pass(p, self.A, self.ws, scales=self.scales, AX=self.AX, YtA=self.YtA)
        ev[2].record()
        gn.gn_core(p, self.AX, out=self.core, ws=self.ws_core, YtA=self.YtA)
        ev[3].record()
        gn.gn_apply(p, 0, self.AX, self.YtA, self.core, self.W, out=self.out)
        ev[4].record()

    def timed(self, steps, warmup):
        import torch
        for _ in range(warmup):
            self.step([torch.cuda.Event(enable_timing=True) for _ in range(5)])
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
        t0 = time.perf_counter()
        for e in evs:
            self.step(e)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = {k: [] for k in ("prepare", "pass", "core", "apply", "step")}
        for e in evs:
            st["prepare"].append(e[0].elapsed_time(e[1]))
            st["pass"].append(e[1].elapsed_time(e[2]))
            st["core"].append(e[2].elapsed_time(e[3]))
            st["apply"].append(e[3].elapsed_time(e[4]))
            st["step"].append(e[0].elapsed_time(e[4]))
        mean = {k: sum(v) / len(v) for k, v in st.items()}
        mean["wall_ms_per_step"] = 1e3 * wall / steps
        return mean

    def error(self):
        """||A - A_hat||_F / ||A||_F on the device, tile by tile, and the kept rank.
        A is the original matrix (for BF16, the FP32 matrix before quantization)."""
        import torch
        gn = self.gn
        F, G = gn.gn_factors(self.p, self.AX, self.YtA, self.core)
        sc = self.scales if self.A_ref is self.A else None
        ss = float(gn.gn_residual(self.A_ref, F, G, scales=sc).item())
        z = torch.zeros(self.w.m, 1, dtype=torch.float64, device="cuda")
        zg = torch.zeros(1, self.w.n, dtype=torch.float64, device="cuda")
        na = float(gn.gn_residual(self.A_ref, z, zg, k=0, scales=sc).item())
        del F, G
        return math.sqrt(ss), math.sqrt(na), self.core.rank(), self.core.flags()


def grad_bench(gn, W, steps=5, warmup=2, host_factors=False):
    """Forward and reverse mode on the gradient workload (8192 x 4096 FP32, sigma_i =
    i^-1.5, Gaussian X and Y, r = 256, l = 128; loss weights Gbar on Philox stream 5).
    The forward is the sketch pass, the core and the materialized A_hat; the
    backward is gn_backward with AX kept from the forward, and with AX recomputed.

    A and Gbar (134 MB each) fit the 256 MB Infinity Cache, so back-to-back calls
    find them there: `*_ms` are such warm calls; `*_cold_ms` time each call alone
    after 1 GiB of writes has evicted the cache (the eviction is outside the timed
    region)."""
    import torch
    wl = W.GRAD8K
    A = W.device_matrix(wl, host_factors=host_factors)
    p = gn.Problem(wl.m, wl.n, wl.r, wl.l, seed=wl.seed, mode="f32", eps=wl.eps)
    Gbar = gn.gn_generate_gaussian(wl.seed, 5, wl.m, wl.n, dtype=torch.float32)
    ws_s, ws_c = gn.workspace(p, gn.C.GN_OP_SKETCH), gn.workspace(p, gn.C.GN_OP_CORE)
    ws_b = gn.workspace(p, gn.C.GN_OP_BACKWARD)
    AX = torch.empty(wl.m, wl.r, dtype=torch.float32, device="cuda")
    YtA = torch.empty(p.rl, wl.n, dtype=torch.float32, device="cuda")
    Ahat = torch.empty(wl.m, wl.n, dtype=torch.float32, device="cuda")
    dA = torch.empty_like(Ahat)
    core = gn.new_core(p)

    def fwd():
        gn.gn_sketch(p, A, AX=AX, YtA=YtA, ws=ws_s)
        gn.gn_core(p, AX, out=core, ws=ws_c, YtA=YtA)
        gn.gn_materialize(p, AX, YtA, core, out=Ahat)

    def bwd(recompute):
        gn.gn_backward(p, Gbar, YtA, core, AX=None if recompute else AX, A=A, dA=dA, ws=ws_b)

    def timeit(f):
        for _ in range(warmup):
            f()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(steps):
            f()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / steps

    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB

    def timeit_cold(f):
        ts = []
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        for _ in range(steps):
            flush.zero_()
            ev[0].record()
            f()
            ev[1].record()
            torch.cuda.synchronize()
            ts.append(ev[0].elapsed_time(ev[1]))
        return sum(ts) / len(ts)

    t_f = timeit(fwd)
    t_b = timeit(lambda: bwd(False))
    t_br = timeit(lambda: bwd(True))
    t_fc = timeit_cold(fwd)
    t_bc = timeit_cold(lambda: bwd(False))
    del flush
    m, n, r, rl = wl.m, wl.n, wl.r, p.rl
    # pass over Gbar and final product 2mn(r + rl) each; H and U = G1 M^T 2m r rl each;
    # V = M^T G2 + Cbar X^T 4 rl n r
    fl_b = 4.0 * m * n * (r + rl) + 2.0 * m * r * rl + 2.0 * m * r * rl + 4.0 * rl * n * r
    fl_f = 2.0 * m * n * (r + rl) + 2.0 * m * r * n
    out = {"workload": wl.name, "m": m, "n": n, "r": r, "l": wl.l, "mode": "f32",
           "kept_rank": core.rank(), "forward_ms": t_f, "backward_ms": t_b,
           "backward_recompute_ax_ms": t_br, "forward_cold_ms": t_fc, "backward_cold_ms": t_bc,
           "infinity_cache": "warm for *_ms (A and Gbar, 134 MB each, stay in the 256 MB "
                             "Infinity Cache between back-to-back calls); evicted before each "
                             "call for *_cold_ms",
           "backward_algorithmic_flops": fl_b,
           "backward_tflops": fl_b / (t_b / 1e3) / 1e12,
           "backward_frac_of_fp32_peak": fl_b / (t_b / 1e3) / 1e12 / PEAK["f32"],
           "forward_algorithmic_flops": fl_f,
           "note": "forward = sketch pass + core + materialized A_hat (F G, 2mnr); "
                   "backward flops = pass over Gbar 2mn(r+rl) + final product 2mn(r+rl) + "
                   "core-size terms"}
    del A, Gbar, AX, YtA, Ahat, dA, ws_s, ws_c, ws_b
    torch.cuda.empty_cache()
    return out


def batch_bench(gn, W, steps=5, warmup=2, count=512, host_factors=False):
    """The batched workload: 512 FP32 problems (m ~ U[256,4096], n ~ U[128,m],
    r ~ U[8,128], l = ceil(r/2), sigma_i = 10^(-8i/n), Gaussian X and Y) solved by
    gn_batch_solve: the pass launch alone, the whole solve, and the
    whole solve replayed from a captured HIP graph."""
    import torch
    from paper_2009_11392_amd.autotune import build_batch_problems
    probs = build_batch_problems(gn, W, count, host_factors=host_factors)
    batch = gn.Batch(probs)
    plan = batch.plan

    def timeit(f):
        for _ in range(warmup):
            f()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(steps):
            f()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / steps

    t_pass = timeit(lambda: batch.solve(gn.C.GN_BATCH_PASS))
    t_solve = timeit(lambda: batch.solve(gn.C.GN_BATCH_ALL))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.solve()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.solve()
    t_graph = timeit(graph.replay)
    ks = [c.rank() for c in batch.core]
    flops, byts = plan.pass_flops, plan.pass_bytes
    out = {"workload": f"batch{count}_f32", "problems": count, "pass_ms": t_pass,
           "solve_ms": t_solve, "graph_solve_ms": t_graph,
           "pass_algorithmic_flops": flops, "pass_algorithmic_bytes": byts,
           "pass_tflops": flops / (t_pass / 1e3) / 1e12,
           "pass_frac_of_fp32_peak": flops / (t_pass / 1e3) / 1e12 / PEAK["f32"],
           "roofline_ms": max(flops / (PEAK["f32"] * 1e12), byts / (HBM_PEAK_GBS * 1e9)) * 1e3,
           "work_items": plan.n_pass_items, "core_items": plan.n_core_items,
           "pass_workgroups": plan.grid, "tile_policy": list(plan.tile_policy),
           "truncated_problems": sum(1 for k, p in zip(ks, batch.problems) if k < p.r),
           "solves_per_sec": count * 1e3 / t_graph}
    del batch, probs, graph
    torch.cuda.empty_cache()
    return out


def stabilize_bench(gn, run, steps=3, warmup=1):
    """The core under each Section 5.1.1 stabilization on the main workload's AX
    (the pass output of the timed steps): truncated QR, the SVD route, the three
    perturbations, and the Section 5.1.2 power-method check of the plain core.
    Each core is timed with HIP events on the library's stream; its approximant's
    error ||A - A_hat||_F / ||A||_F is measured on the device."""
    import dataclasses
    import torch

    def timeit(f):
        for _ in range(warmup):
            f()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(steps):
            f()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / steps

    z = torch.zeros(run.w.m, 1, dtype=torch.float64, device="cuda")
    zg = torch.zeros(1, run.w.n, dtype=torch.float64, device="cuda")
    na = math.sqrt(float(gn.gn_residual(run.A, z, zg, k=0, scales=run.scales).item()))
    out = {"workload": run.w.name, "r": run.w.r, "l": run.p.l_eff, "methods": {}}
    for method in ("qr", "svd", "lift_svd", "lift_rrqr", "lift_diag"):
        p = dataclasses.replace(run.p, core_method=method)
        ws = gn.workspace(p, gn.C.GN_OP_CORE)
        core = gn.new_core(p)
        ms = timeit(lambda: gn.gn_core(p, run.AX, out=core, ws=ws, YtA=run.YtA))
        F, G = gn.gn_factors(p, run.AX, run.YtA, core)
        e = math.sqrt(float(gn.gn_residual(run.A, F, G, scales=run.scales).item()))
        out["methods"][method] = {"core_ms": ms, "kept_rank": core.rank(),
                                  "status_flags": core.flags(), "rel_err": e / na}
        log(f"core {method}: {ms:.2f} ms, k={core.rank()}, flags={core.flags()}, err {e / na:.4e}")
        del F, G, ws, core
        torch.cuda.empty_cache()
    plain = dataclasses.replace(run.p, eps=0.0, core_method="qr")
    core = gn.gn_core(plain, run.AX, YtA=run.YtA)
    est = torch.zeros(1, dtype=torch.float64, device="cuda")
    ms = timeit(lambda: gn.gn_core_check(plain, core, run.p.eps, 8, 4, est=est))
    out["check"] = {"ms": ms, "start_vectors": 8, "iterations": 4,
                    "estimate_inv_norm": float(est.item()), "flagged": bool(core.flags() & 8),
                    "delta": run.p.eps}
    log(f"check of the plain core: {ms:.3f} ms, estimate {float(est.item()):.3e}, "
        f"flagged={bool(core.flags() & 8)}")
    return out


def r_sweep(gn, W, A32, steps=3, warmup=1,
            rs=(4, 8, 16, 32, 64, 128, 256, 512, 1000, 2000)):
    """The sketch pass alone on the 32768^2 matrix with Gaussian X and Y over r
    (l = ceil(r/2)), in FP32 and in BF16 with block scales: the pass is bound by
    HBM bandwidth at small r (about r < 16 in FP32, r < 125 in BF16) and by the
    matrix cores above; each point reports its algorithmic bytes and flops, the
    bound, the achieved rate and the fraction of that bound's peak."""
    import torch
    out = {"shape": "32768x32768, Gaussian X and Y, l = ceil(r/2)", "points": []}
    for mode, base in (("f32", W.F32_32K), ("bf16", W.BF16_32K)):
        if mode == "bf16":
            A, sc = gn.gn_quantize_bf16_bs(A32)
        else:
            A, sc = A32, None
        for r in rs:
            wl = base.scaled(base.m, base.n, r=r)
            p = gn.Problem(wl.m, wl.n, wl.r, wl.l, seed=wl.seed, mode=mode, eps=wl.eps)
            ws = gn.workspace(p, gn.C.GN_OP_SKETCH)
            AX = torch.empty(wl.m, wl.r, dtype=torch.float32, device="cuda")
            YtA = torch.empty(p.rl, wl.n, dtype=torch.float32, device="cuda")
            gn.gn_sketch_prepare(p, ws)
            for _ in range(warmup):
                gn.gn_sketch_pass(p, A, ws, scales=sc, AX=AX, YtA=YtA)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            for _ in range(steps):
                gn.gn_sketch_pass(p, A, ws, scales=sc, AX=AX, YtA=YtA)
            ev[1].record()
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / steps
            fl, by = pass_algorithmic(wl, srht_pad(wl.n))
            t_hbm, t_mma = by / (HBM_PEAK_GBS * 1e9), fl / (PEAK[mode] * 1e12)
            bound = "hbm" if t_hbm >= t_mma else "mfma"
            ach = by / (ms / 1e3) / 1e9 if bound == "hbm" else fl / (ms / 1e3) / 1e12
            peak = HBM_PEAK_GBS if bound == "hbm" else PEAK[mode]
            pt = {"mode": mode, "r": r, "l": wl.l, "pass_ms": ms, "algorithmic_bytes": by,
                  "algorithmic_flops": fl, "bound": bound, "achieved": ach,
                  "unit": "GB/s" if bound == "hbm" else "TFLOP/s", "peak": peak,
                  "frac": ach / peak, "gbps": by / (ms / 1e3) / 1e9,
                  "tflops": fl / (ms / 1e3) / 1e12}
            out["points"].append(pt)
            log(f"r-sweep {mode} r={r}: {ms:.3f} ms, {pt['gbps']:.0f} GB/s, "
                f"{pt['tflops']:.1f} TFLOP/s, {bound} frac {pt['frac']:.3f}")
            del ws, AX, YtA
        del A, sc
        torch.cuda.empty_cache()
    return out


def host_threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def oracle_sketches(w, workers):
    """The oracle's X and Y for workload w, holding the values the working
    precision stores (an SRHT X is the explicit +-1 matrix)."""
    from oracle import gn as OG, philox as OP
    mode = "f64" if w.mode == "f64" else w.mode
    if w.kind_x == "srht":
        X = OP.srht_matrix(w.seed, w.n, w.r)
    else:
        X = OG.round_mode(OP.gaussian(w.seed, OP.STREAM_X, w.n, w.r, workers=workers), mode)
    Y = OG.round_mode(OP.gaussian(w.seed, OP.STREAM_Y, w.m, w.r + w.l, workers=workers), mode)
    return X, Y


def oracle_tau(w):
    from oracle import gn as OG
    nx = OG.nu_srht(w.n) if w.kind_x == "srht" else OG.nu_gaussian(w.n, w.r)
    return OG.threshold(w.eps, nx, OG.nu_gaussian(w.m, w.r + w.l))


def cpu_baseline(A_dev, w, npad):
    """The FP64 oracle's whole GN solve of the workload on the host cores: the
    sketches, the sketch pass A@X and Y^T@A (timed: `value`), the core and the
    factors (timed with the pass: `solve_seconds`), then ||A - A_hat||_F (not
    timed) for the error ratio of the GPU solve."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import gn as OG

    workers = host_threads()
    A64 = A_dev.cpu().numpy().astype(np.float64)
    X, Y = oracle_sketches(w, workers)
    t0 = time.perf_counter()
    AX, YA = OG.sketch_pass(A64, X, Y)
    t1 = time.perf_counter()
    c = OG.core(AX, Y, oracle_tau(w))
    F, G = OG.factors(AX, YA, c)
    t2 = time.perf_counter()
    e = OG.residual_fro(A64, F, G)
    na = float(np.linalg.norm(A64))
    flops, _ = pass_algorithmic(w, npad)
    threads = max([d.get("num_threads", 0) for d in threadpool_info()] or [os.cpu_count() or 1])
    dense = " (A@X as a dense product with the explicit +-1 SRHT matrix, 2mnr flops)" \
        if w.kind_x == "srht" else ""
    return {"value": flops / (t1 - t0) / 1e12, "unit": "TFLOP/s", "cores": int(threads),
            "kind": "oracle",
            "sample": (f"FP64 NumPy oracle, whole {w.m}x{w.n} matrix: the sketch pass A@X, "
                       f"Y^T@A timed ({t1 - t0:.2f} s){dense}; value = the method's "
                       f"algorithmic pass flops / that time, as for the GPU value"),
            "seconds": t1 - t0, "solve_seconds": t2 - t0, "kept_rank": c.k,
            "abs_err": e, "rel_err": e / na}


def oracle_error(A_dev, w):
    """||A - A_hat||_F of the FP64 oracle's GN on A_dev (as FP64) with workload w's
    sketch values (not timed)."""
    import numpy as np

    from oracle import gn as OG

    A64 = A_dev.cpu().numpy().astype(np.float64)
    X, Y = oracle_sketches(w, host_threads())
    res = OG.gn(A64, X, Y, oracle_tau(w))
    e = OG.residual_fro(A64, res.F, res.G)
    return e, e / float(np.linalg.norm(A64)), res.core.k


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="srht_32768x32768_f32")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--no-grad", action="store_true", help="skip the reverse-mode measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-workload measurement")
    ap.add_argument("--no-small-r", action="store_true",
                    help="skip the small-r (HBM-bound) pass measurement")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the r-sweep of the sketch pass (FP32 and BF16, r = 4 .. 2000)")
    ap.add_argument("--no-stab", action="store_true",
                    help="skip the timing of the other core stabilizations and the check")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (reference for HBM counters)")
    ap.add_argument("--host-factors", action="store_true",
                    help="build the test matrix's orthonormal factors on the host (no library "
                         "kernels on the device; used for hardware-counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the library runs the path on a single MI355X).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2009_11392_amd import gn, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    gn.C.lib()  # fail loudly if the library is not built
    w = W.ALL[args.workload]
    npad = srht_pad(w.n)
    log(f"generating {w.name} on the device")
    A32 = W.device_matrix(w if w.mode not in ("bf16", "f16") else W.F32_32K,
                          host_factors=args.host_factors)
    scales = None
    if w.mode == "bf16":
        A, scales = gn.gn_quantize_bf16_bs(A32)
    elif w.mode == "f16":
        A, scales = gn.gn_quantize_f16_bs(A32)
    elif w.mode == "f64":
        A = A32.double()
    else:
        A = A32
    torch.cuda.synchronize()

    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: 3 x 1 GiB device-to-device")

    run = Runner(gn, w, A, scales)
    log(f"timing {args.steps} steps after {args.warmup} warm-up steps")
    t = run.timed(args.steps, args.warmup)
    flops, byts = pass_algorithmic(w, npad)
    pass_s = t["pass"] / 1e3
    tflops = flops / pass_s / 1e12
    gbs = byts / pass_s / 1e9
    solve_ms = t["prepare"] + t["pass"] + t["core"]
    peak = PEAK[w.mode]
    bound = "mfma" if flops / (peak * 1e12) > byts / (HBM_PEAK_GBS * 1e9) else "hbm"
    roof = {"bound": bound, "kernel": "fused sketch pass (gn_sketch_pass)",
            "achieved": tflops if bound == "mfma" else gbs, "peak": peak if bound == "mfma" else HBM_PEAK_GBS,
            "unit": "TFLOP/s" if bound == "mfma" else "GB/s",
            "traffic": traffic_from_profile(w.name),
            "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": byts,
            "avg_launch_ms": t["pass"]}
    roof["frac"] = roof["achieved"] / roof["peak"]
    res = {"metric": METRIC, "value": tflops, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": t["step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": w.mode,
           "data": "synthetic (seeded spectrum-controlled matrix generated on the device)",
           "config": {"workload": w.name, "m": w.m, "n": w.n, "r": w.r, "l": w.l,
                      "sketch_x": w.kind_x, "sketch_y": w.kind_y, "pass_precision": w.mode,
                      "core_precision": "f64", "parallelism": "single GPU"},
           "pass_gbps": gbs, "pass_ms": t["pass"], "solves_per_sec": 1e3 / solve_ms,
           "stage_ms": {k: t[k] for k in ("prepare", "pass", "core", "apply")},
           "wall_ms_per_step": t["wall_ms_per_step"], "roofline": roof}
    log(f"pass {t['pass']:.3f} ms  {tflops:.1f} TFLOP/s  {gbs:.0f} GB/s  solve {solve_ms:.2f} ms")

    if not args.no_error:
        e, na, k, flags = run.error()
        res["error"] = {"rel_fro": e / na, "abs_fro": e, "kept_rank": k, "status_flags": flags,
                        "optimum_estimate": optimum_estimate(w),
                        "ratio_to_optimum": e / optimum_estimate(w)}
        log(f"error {e / na:.4e} (abs {e:.4e}, k={k})")

    if not args.no_stab:
        log("core stabilizations and the plain-GN check")
        res["stabilizations"] = stabilize_bench(gn, run)

    if not args.no_small_r and w is W.SRHT32K:
        # the same resident matrix at r = 10, l = 5: the pass is then bound by
        # HBM bandwidth (45 flops per 4-byte element), not by the matrix cores
        ws_ = W.SRHT32K_R10
        log(f"small r: {ws_.name}")
        rs = Runner(gn, ws_, A)
        ts = rs.timed(20, 3)
        fl, by = pass_algorithmic(ws_, npad)
        gb = by / (ts["pass"] / 1e3) / 1e9
        res["small_r"] = {"workload": ws_.name, "r": ws_.r, "l": ws_.l, "pass_ms": ts["pass"],
                          "bound": "hbm", "achieved_gbps": gb, "peak_gbps": HBM_PEAK_GBS,
                          "frac": gb / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": by,
                          "traffic": traffic_from_profile(ws_.name),
                          "solves_per_sec": 1e3 / (ts["prepare"] + ts["pass"] + ts["core"])}
        log(f"small r pass {ts['pass']:.3f} ms  {gb:.0f} GB/s ({gb / HBM_PEAK_GBS:.3f} of HBM peak)")
        del rs

    if not args.no_compare and w.m == 32768 and w.n == 32768:
        cmp = {}
        for tag, wl in (("bf16", W.BF16_32K), ("f16", W.F16_32K), ("f32", W.F32_32K)):
            log(f"comparison: {wl.name}")
            if tag == "bf16":
                Ab, sc = gn.gn_quantize_bf16_bs(A32)
            elif tag == "f16":
                Ab, sc = gn.gn_quantize_f16_bs(A32)
            else:
                Ab, sc = A32, None
            rr = Runner(gn, wl, Ab, sc, A_ref=A32)
            tt = rr.timed(3, 1)
            fl, by = pass_algorithmic(wl, srht_pad(wl.n))
            ent = {"pass_ms": tt["pass"], "solve_ms": tt["prepare"] + tt["pass"] + tt["core"],
                   "pass_tflops": fl / (tt["pass"] / 1e3) / 1e12,
                   "pass_frac_of_peak": fl / (tt["pass"] / 1e3) / 1e12 / PEAK[tag],
                   "pass_algorithmic_bytes": by, "pass_traffic": traffic_from_profile(wl.name)}
            ent["solves_per_sec"] = 1e3 / ent["solve_ms"]
            e, na, k, flags = rr.error()
            ent.update({"rel_err": e / na, "abs_err": e, "kept_rank": k, "status_flags": flags})
            cmp[tag] = ent
            del rr, Ab
            torch.cuda.empty_cache()
        cmp["speedup_solves_per_sec"] = cmp["bf16"]["solves_per_sec"] / cmp["f32"]["solves_per_sec"]
        cmp["speedup_pass"] = cmp["f32"]["pass_ms"] / cmp["bf16"]["pass_ms"]
        cmp["err_ratio_bf16_over_f32"] = cmp["bf16"]["rel_err"] / cmp["f32"]["rel_err"]
        cmp["f16_speedup_solves_per_sec"] = cmp["f16"]["solves_per_sec"] / cmp["f32"]["solves_per_sec"]
        cmp["f16_speedup_pass"] = cmp["f32"]["pass_ms"] / cmp["f16"]["pass_ms"]
        cmp["err_ratio_f16_over_f32"] = cmp["f16"]["rel_err"] / cmp["f32"]["rel_err"]
        cmp["shape"] = "32768x32768, Gaussian X and Y, r=2000, l=1000, same matrix"
        res["bf16_vs_fp32"] = cmp

    if not args.no_sweep and w.m == 32768 and w.n == 32768:
        log("r-sweep of the sketch pass (FP32 and BF16, Gaussian X and Y)")
        res["r_sweep"] = r_sweep(gn, W, A32)

    if not args.no_grad:
        log("reverse mode: grad_8192x4096_f32")
        res["gradient"] = grad_bench(gn, W, host_factors=args.host_factors)
        log(f"forward {res['gradient']['forward_ms']:.3f} ms, backward "
            f"{res['gradient']['backward_ms']:.3f} ms "
            f"({res['gradient']['backward_tflops']:.1f} TFLOP/s)")

    if not args.no_batch:
        log("batched workload: 512 problems")
        res["batched"] = batch_bench(gn, W, host_factors=args.host_factors)
        log(f"batched pass {res['batched']['pass_ms']:.3f} ms "
            f"({res['batched']['pass_tflops']:.1f} TFLOP/s), solve {res['batched']['solve_ms']:.3f} ms, "
            f"graph {res['batched']['graph_solve_ms']:.3f} ms")

    if not args.no_cpu:
        log("cpu baseline: the FP64 oracle's solve of the same matrix on the host")
        cb = cpu_baseline(A32 if w.mode != "f64" else A, w, npad)
        res["cpu_baseline"] = cb
        log(f"oracle pass {cb['seconds']:.2f} s ({cb['value']:.3f} TFLOP/s, {cb['cores']} threads), "
            f"rel err {cb['rel_err']:.6e}")
        if "error" in res:
            res["error"]["oracle_rel_err"] = cb["rel_err"]
            res["error"]["oracle_kept_rank"] = cb["kept_rank"]
            res["error"]["err_ratio_vs_oracle"] = res["error"]["abs_fro"] / cb["abs_err"]
            log(f"error ratio vs the FP64 oracle: {res['error']['err_ratio_vs_oracle']:.6f}")
        if "bf16_vs_fp32" in res:
            for tag, wl in (("bf16", W.BF16_32K), ("f16", W.F16_32K)):
                log(f"FP64 oracle on the {tag} variant's sketch values (unquantized matrix)")
                eo, ro, ko = oracle_error(A32, wl)
                b = res["bf16_vs_fp32"][tag]
                b.update({"oracle_rel_err": ro, "oracle_kept_rank": ko,
                          "err_ratio_vs_oracle": b["abs_err"] / eo})
                log(f"{tag} error ratio vs the FP64 oracle: {b['err_ratio_vs_oracle']:.6f}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
