#!/usr/bin/env python3
"""Throughput of the WarpLDA sweep on one MI355X.

A step is one full iteration (word phase + document phase) of the sampler over
the whole synthetic corpus, already resident in HBM.  Default workload: the
NYTimes-shaped corpus (D=300k, V=100k, Zipf(1.0) words, lognormal(mean 330,
sigma 0.8) doc lengths, ~99M tokens) with K=1000, alpha=50/K, beta=0.01, M=2.

Prints ONE JSON line.  Besides the throughput it reports the roofline of the
kernel that takes the most time (algorithmic bytes of one launch over its
average duration, timed with HIP events on the sampler's stream during the
timed steps) and the single-threaded CPU oracle timed on a bounded sample of
the same corpus.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes_per_token(kind: str, M: int) -> float:
    """Bytes the method itself moves per token (int32 topics): a word phase
    reads and writes z and the M proposals (8 + 8M); a document phase also
    reads one row pointer (12 + 8M).  The multi-workgroup path splits the
    phase over three kernels: histogram (reads z), MH (reads z and the M
    proposals, writes z) and draw (writes the M proposals)."""
    extra = 4.0 if kind.startswith("doc") else 0.0
    if kind.endswith("_hist"):
        return 4.0 + extra
    if kind.endswith("_mh"):
        return 4.0 * (1 + M) + 4.0 + extra
    if kind.endswith("_draw"):
        return 4.0 * M + extra
    return 8.0 + 8.0 * M + extra


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1510_08628_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1510_08628_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(c, wl, n_docs: int, iters: int):
    import oracle
    import synth
    p = synth.doc_prefix(c, n_docs)
    o = oracle.Oracle(p.word_ids, p.doc_ids, p.V, p.D, wl.K, wl.M, wl.alpha, wl.beta, seed=1)
    o.init()
    o.iterate(1)                       # warm-up
    t0 = time.perf_counter()
    o.iterate(iters)
    dt = time.perf_counter() - t0
    return {"value": p.T * iters / dt, "unit": "tokens/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_docs} docs of the same corpus ({p.T} tokens, V={p.V}), "
                      f"{iters} iterations after 1 warm-up, single thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="nytimes-shape-k1e3")
    ap.add_argument("--M", type=int, default=None, help="override the MH steps")
    ap.add_argument("--cpu-docs", type=int, default=30000)
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_1510_08628_amd as W

    W.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = synth.WORKLOADS[args.workload]
    M = args.M or wl.M
    t0 = time.perf_counter()
    c = wl.make()
    log(f"[bench] corpus {args.workload}: T={c.T} V={c.V} D={c.D} ({time.perf_counter() - t0:.1f}s)")

    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib << 20
        a = torch.empty(n, dtype=torch.uint8, device=dev)
        b = torch.empty(n, dtype=torch.uint8, device=dev)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {n} bytes done")
        del a, b

    t0 = time.perf_counter()
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, wl.K, M, wl.alpha, wl.beta, seed=1, device=dev)
    s.init()
    torch.cuda.synchronize()
    log(f"[bench] create+init {time.perf_counter() - t0:.1f}s, workspace {s.workspace_bytes / 2**30:.2f} GiB")

    s.iterate(args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] warm-up {args.warmup} iterations done")
    s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = s.profile_read()
    s.profile(False)
    log(f"[bench] timed {args.steps} iterations in {dt * 1e3:.2f} ms")

    kernels = {}
    for name, (launches, tokens, total_ms) in stats.items():
        if launches == 0:
            continue
        avg = total_ms / launches
        bpt = algorithmic_bytes_per_token(name, M)
        kernels[name] = dict(avg_ms=avg, tokens=tokens, gbps=bpt * tokens / (avg * 1e-3) / 1e9)
        log(f"[bench]   {name:16s} {avg:8.4f} ms/launch  {tokens:>11d} tokens  "
            f"{kernels[name]['gbps']:8.1f} GB/s algorithmic")
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    achieved = kernels[dom]["gbps"]
    traffic = measured_traffic(args.workload, dom)
    iter_bytes = (20 + 16 * M) * c.T
    log(f"[bench] iteration algorithmic rate {iter_bytes * args.steps / dt / 1e9:.1f} GB/s, "
        f"LL={s.log_likelihood():.6e}")

    out = {
        "metric": "sampled tokens/s/GPU",
        "value": c.T * args.steps / dt,
        "unit": "tokens/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "tokens": c.T, "V": c.V, "D": c.D, "K": wl.K,
                   "M": M, "alpha": wl.alpha, "beta": wl.beta, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
    }
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(c, wl, args.cpu_docs, args.cpu_iters)
        log(f"[bench] cpu baseline {time.perf_counter() - t0:.1f}s")
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
