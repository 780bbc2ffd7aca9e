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


# --------------------------------------------------------------------------
# Learned proposal + serving (fold-in of new documents against the fit)
# --------------------------------------------------------------------------
SWEEP_GRID = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 200]


def train_encoder(W, s, c, wl, dev, epochs, batch, hidden=512, buckets=100_000, lr=1e-3,
                  w1_std=0.25):
    """Adam on the sampler's own (document, theta_hat_d) pairs."""
    import numpy as np
    import torch
    import synth
    t0 = time.perf_counter()
    counts = np.bincount(c.doc_ids, minlength=c.D)
    docptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint64)
    order = np.argsort(c.doc_ids, kind="stable")
    rowptr, idx, val = W.features_csr(buckets, docptr, c.word_ids[order])
    d_rp = torch.from_numpy(rowptr.astype(np.int32)).to(dev)
    d_idx = torch.from_numpy(idx.astype(np.int32)).to(dev)
    d_val = torch.from_numpy(val).to(dev)
    theta = s.theta(0, c.D)
    enc = W.Encoder(buckets, hidden, wl.K, max_batch=batch, lr=lr, device=dev)
    enc.set_weights(synth.encoder_init_weights(buckets, hidden, wl.K, 11, w1_std))
    t_feat = time.perf_counter() - t0
    losses = []
    t1 = time.perf_counter()
    steps = 0
    for ep in range(epochs):
        for b0 in range(0, c.D - batch + 1, batch):
            want = (steps % 200) == 0
            l = enc.train_step(d_rp[b0:b0 + batch + 1], d_idx, d_val, theta[b0:b0 + batch], want)
            if want:
                losses.append(l)
            steps += 1
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    # the floor of the soft cross-entropy: mean entropy of the targets
    th = theta[:4096].double()
    ent = float(-(th * th.log()).sum(1).mean())
    log(f"[serve] encoder: features {t_feat:.1f}s, {steps} steps in {t_train:.1f}s, "
        f"loss {losses[0]:.4f} -> {losses[-1]:.4f} (target entropy {ent:.4f})")
    del theta
    return enc, dict(steps=steps, train_s=t_train, loss_first=losses[0], loss_last=losses[-1],
                     target_entropy=ent, epochs=epochs, batch=batch, hidden=hidden,
                     buckets=buckets)


def encoder_weights(W, enc, docptr, words, dev, eps=0.01):
    """Learned-proposal weights (n x K) of documents from the encoder."""
    import numpy as np
    import torch
    rowptr, idx, val = W.features_csr(enc.buckets, docptr, words)
    n = len(docptr) - 1
    d_idx = torch.from_numpy(idx.astype(np.int32)).to(dev)
    d_val = torch.from_numpy(val).to(dev)
    out = []
    for b0 in range(0, n, enc.max_batch):
        b1 = min(n, b0 + enc.max_batch)
        rp = torch.from_numpy((rowptr[b0:b1 + 1]).astype(np.int32)).to(dev)
        probs = enc.forward(rp, d_idx, d_val)
        cdf = enc.proposal(probs, eps).cpu().numpy().astype(np.int64)
        out.append(np.diff(np.concatenate([np.zeros((b1 - b0, 1), np.int64), cdf], 1), axis=1))
    return np.concatenate(out).astype(np.uint32)


def foldin_curve(gm, docptr, words, req, hoptr, how, weights=None, ls=0):
    """Total held-out LL after S sweeps, for S on SWEEP_GRID."""
    curve = {}
    for S in SWEEP_GRID:
        _, ho = gm.foldin(docptr, words, req, S, weights, ls, hoptr, how)
        curve[S] = float(ho.sum())
    return curve


def sweeps_to(curve, ref_ll, tol):
    """Smallest S on the grid whose held-out LL is within tol (relative) of ref_ll."""
    for S in SWEEP_GRID:
        if abs(curve[S] - ref_ll) <= tol * abs(ref_ll):
            return S
    return None


def serve(W, gm, enc, docptr, words, hoptr, how, arrivals, sweeps, weights=None, ls=2):
    import numpy as np
    n = len(docptr) - 1
    srv = W.Server(gm, enc, max_docs=2048, pool_tokens=4 << 20, pool_heldout=4 << 20,
                   sweeps=sweeps, learned_steps=ls)
    t0 = srv.now()
    nxt, done, lat, ll, steps = 0, 0, [], 0.0, 0
    tokens = int(docptr[-1])
    while done < n:
        now = srv.now() - t0
        while nxt < n and arrivals[nxt] <= now:
            a, b = int(docptr[nxt]), int(docptr[nxt + 1])
            h0, h1 = int(hoptr[nxt]), int(hoptr[nxt + 1])
            srv.submit(nxt, words[a:b], how[h0:h1], arrival=t0 + arrivals[nxt],
                       weights=None if weights is None else weights[nxt])
            nxt += 1
        srv.step()
        steps += 1
        for r in srv.poll():
            lat.append(r["done_s"] - r["arrival_s"])
            ll += r["heldout_ll"]
            srv.take_z(r["req_id"], r["n_tokens"])
            done += 1
    wall = srv.now() - t0
    lat = np.array(lat) * 1e3
    srv.close()
    return dict(sweeps=sweeps, p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()),
                docs_per_s=n / wall, tokens_per_s=tokens / wall, heldout_ll=ll, steps=steps)


def serving_experiment(W, dev, n_eval=1000, n_req=4000, rate=2000.0, epochs=3, batch=256,
                       fit_iters=1000, workload="nytimes-shape-topical-k1e3"):
    """Learned vs plain fold-in against a model frozen from a K=1000 fit.

    The fit runs on the topical variant of the NYTimes-shaped corpus (same
    D, V, lengths and Zipf(1.0) word frequencies, but LDA-generated with
    Zipf-shaped topics): an iid-Zipf corpus has no topics to fold in against.
    New documents are drawn from the fitted model and split 50/50 into
    observed and held-out tokens.  S* is the fewest sweeps whose held-out LL
    is within 1% (and within 0.1%) of a 200-sweep plain chain; the server then
    runs Poisson arrivals at `rate` at each chain's S* (0.1%)."""
    import numpy as np
    import torch
    import synth
    t0 = time.perf_counter()
    wl = synth.WORKLOADS[workload]
    c = wl.make()
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, wl.K, wl.M, wl.alpha, wl.beta, seed=1,
                  device=dev)
    s.init()
    s.iterate(fit_iters)
    torch.cuda.synchronize()
    fit_ll = s.log_likelihood()
    log(f"[serve] {workload}: T={c.T}, fit {fit_iters} iterations, LL {fit_ll:.6e} "
        f"({time.perf_counter() - t0:.1f}s)")
    z, _ = s.assignments()
    gm = W.Model(c.word_ids, c.doc_ids, z, c.V, c.D, wl.K, s.M, wl.alpha, wl.beta, seed=5,
                 device=dev)
    enc, enc_stats = train_encoder(W, s, c, wl, dev, epochs, batch, lr=2e-3, w1_std=1.0)
    s.close()
    ev = synth.docs_from_model(c.word_ids, z, c.V, wl.K, wl.alpha, wl.beta, n_eval, 31)
    rq = synth.docs_from_model(c.word_ids, z, c.V, wl.K, wl.alpha, wl.beta, n_req, 32)
    del z
    req = np.arange(n_eval, dtype=np.uint32)
    c_plain = foldin_curve(gm, ev[0], ev[1], req, ev[2], ev[3])
    ref = c_plain[200]
    w_ev = encoder_weights(W, enc, ev[0], ev[1], dev)
    c_learn = foldin_curve(gm, ev[0], ev[1], req, ev[2], ev[3], w_ev, 2)
    star = {f"{tol:g}": {"plain": sweeps_to(c_plain, ref, tol),
                         "learned": sweeps_to(c_learn, ref, tol)} for tol in (0.01, 0.001)}
    log(f"[serve] reference LL (200 plain sweeps) {ref:.1f}; sweeps to target: {star}")
    log(f"[serve] plain curve   {c_plain}")
    log(f"[serve] learned curve {c_learn}")
    arrivals = synth.poisson_arrivals(n_req, rate, 33)
    res = {"workload": workload, "fit_iterations": fit_iters, "fit_ll": fit_ll,
           "reference_ll_200_plain": ref, "eval_docs": n_eval, "requests": n_req,
           "arrival_rate_per_s": rate, "encoder": enc_stats, "sweeps_to_target": star,
           "curve_plain": c_plain, "curve_learned": c_learn}
    sp, sl = star["0.001"]["plain"], star["0.001"]["learned"]
    if sp is not None:
        res["plain"] = serve(W, gm, None, rq[0], rq[1], rq[2], rq[3], arrivals, sp)
        log(f"[serve] plain   {res['plain']}")
    if sl is not None:
        res["learned"] = serve(W, gm, enc, rq[0], rq[1], rq[2], rq[3], arrivals, sl)
        log(f"[serve] learned {res['learned']}")
    res["total_s"] = time.perf_counter() - t0
    enc.close()
    gm.close()
    return res


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
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the learned-proposal fold-in / serving measurement")
    ap.add_argument("--serve-requests", type=int, default=4000)
    ap.add_argument("--fit-iters", type=int, default=None,
                    help="iterations of the fit that the fold-in model is frozen from")
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
    if not args.no_serving:
        s.close()
        del s
        out["serving"] = serving_experiment(W, dev, n_req=args.serve_requests,
                                            fit_iters=args.fit_iters or 1000)
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(c, wl, args.cpu_docs, args.cpu_iters)
        log(f"[bench] cpu baseline {time.perf_counter() - t0:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
