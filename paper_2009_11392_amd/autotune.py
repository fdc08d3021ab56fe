"""Tile-policy autotuner for batched solves.

    python -m paper_2009_11392_amd.autotune [--count 512] [--out tile_table.json]

Builds the batched workload (the same seeded problems the benchmark uses), times
the sketch-pass launch of gn_batch_solve for every candidate tile
policy (which 256-thread MFMA tile each product uses: Y^T A with r + l <= 64 or
> 64, AX with r <= 64 or > 64) and writes the fastest to the table that
gn.Batch reads by default.  Timing only: every policy computes the same products.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tile_table.json")

# candidate tile configurations per slot (rows x columns): 256-thread workgroups
# 0 = 64 x 256, 1 = 128 x 128, 2 = 256 x 64; 512-thread workgroups 3 = 128 x 256,
# 4 = 256 x 128.  One launch uses one workgroup size.
CANDIDATES_256 = ([0, 1], [1, 0, 2], [2, 1], [1, 2])
CANDIDATES_512 = ([3, 4], [3, 4], [4, 3], [4, 3])


def load_policy(key: str = "batch_f32"):
    """The tuned policy for `key`, or None when no table has been written."""
    if not os.path.exists(TABLE):
        return None
    with open(TABLE) as f:
        ent = json.load(f).get(key)
    return None if ent is None else list(ent["policy"])


def build_batch_problems(gn, W, count: int, host_factors: bool = False):
    probs = []
    for b in W.batch_specs(count):
        A = W.batch_device_matrix(b, host_factors=host_factors)
        p = gn.Problem(b.m, b.n, b.r, b.l, seed=b.seed, mode="f32",
                       eps=10 * 2.0 ** -24 * float(b.sigma()[0]))
        probs.append((p, A))
    return probs


def time_pass(gn, batch, reps: int = 5) -> float:
    import torch
    batch.solve(gn.C.GN_BATCH_PASS)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        batch.solve(gn.C.GN_BATCH_PASS)
    ev[1].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) / reps


def tune(count: int = 512, out: str = TABLE):
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2009_11392_amd import gn, workloads as W
    assert torch.cuda.is_available(), "the autotuner measures on the GPU"
    probs = build_batch_problems(gn, W, count)
    results = []
    for pol in itertools.chain(itertools.product(*CANDIDATES_256),
                               itertools.product(*CANDIDATES_512)):
        batch = gn.Batch(probs, tile_policy=pol)
        ms = time_pass(gn, batch)
        results.append({"policy": list(pol), "pass_ms": ms,
                        "tflops": batch.plan.pass_flops / (ms / 1e3) / 1e12})
        print(f"[autotune] policy {pol}: {ms:.3f} ms ({results[-1]['tflops']:.1f} TFLOP/s)",
              file=sys.stderr, flush=True)
        del batch
        torch.cuda.empty_cache()
    best = min(results, key=lambda e: e["pass_ms"])
    table = {}
    if os.path.exists(out):
        with open(out) as f:
            table = json.load(f)
    table["batch_f32"] = {"policy": best["policy"], "pass_ms": best["pass_ms"],
                          "problems": count, "candidates": results,
                          "device": torch.cuda.get_device_name(0),
                          "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    best = tune(args.count, args.out)
    print(json.dumps(best))


if __name__ == "__main__":
    main()
