#!/usr/bin/env python3
"""Throughput of the WarpLDA sweep on one MI355X.

A step is one full iteration (word phase + document phase) of the sampler over
the whole synthetic corpus, already resident in HBM.  Default workload: the
NYTimes-shaped corpus (D=300k, V=100k, Zipf(1.0) words, lognormal(mean 330,
sigma 0.8) doc lengths, ~99M tokens) with K=1000, alpha=50/K, beta=0.01, M=2.

Prints ONE JSON line.  Besides the throughput it reports the roofline of the
kernel that takes the most time (algorithmic bytes of one launch over its
average duration, timed with HIP events on the sampler's stream during the
timed steps) and of the whole sweep; the same figures for the other
single-GPU workloads (PubMed-shaped at K=1e4, M=4 and M=2, full size; the
first 2M documents of the ClueWeb-shaped share at K=1e6); the learned vs plain
fold-in experiment with its serving latencies; and the single-threaded CPU
oracle timed on bounded samples of the same corpora.
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
    reads one row pointer (12 + 8M).  The multi-workgroup path splits a phase
    over three kernels, charged so that they sum to the same figure: the
    histogram pass reads z (and the row pointer), the MH pass reads the M
    proposals and writes z, the draw pass writes the M proposals.  Its extra
    reads of z (the MH and draw passes read it again) are traffic, not
    algorithmic bytes."""
    extra = 4.0 if kind.startswith("doc") else 0.0
    if kind.endswith("_hist"):
        return 4.0 + extra
    if kind.endswith("_mh"):
        return 4.0 * M + 4.0
    if kind.endswith("_draw"):
        return 4.0 * M
    return 8.0 + 8.0 * M + extra


# The sources of the sweep's kernels and their launches: a traffic summary
# taken on other versions of these does not describe the current kernels.
SWEEP_SOURCES = ("wlda_device.h", "wlda_host.cpp", "wlda_internal.h", "wlda_kernels.hip",
                 "wlda_kernels_impl.h", "wlda_kernels_m.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
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


def cpu_info() -> dict:
    """Host cores and CPU model of the machine the oracle is timed on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"nproc": os.cpu_count(), "cpus_available": avail, "cpu_model": model}


def oracle_rate(c, wl, M, iters, warmup):
    """Tokens/s of the single-threaded oracle: iters iterations after init and
    warmup iterations."""
    import oracle
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, wl.K, M, wl.alpha, wl.beta, seed=1)
    o.init()
    if warmup:
        o.iterate(warmup)
    t0 = time.perf_counter()
    o.iterate(iters)
    dt = time.perf_counter() - t0
    return c.T * iters / dt, dt


def cpu_baseline(c1, args):
    """The oracle as it stands, single thread, on bounded samples: the first
    docs of the NYTimes-shaped corpus (the headline value), and per workload
    the whole tiny LDA corpus (50 iterations), and document prefixes of the
    PubMed-shaped and ClueWeb-shaped corpora (1 iteration each)."""
    import synth
    info = cpu_info()
    wl1 = synth.WORKLOADS["nytimes-shape-k1e3"]
    p = synth.doc_prefix(c1, args.cpu_docs)
    rate, dt = oracle_rate(p, wl1, wl1.M, args.cpu_iters, 1)
    out = {"value": rate, "unit": "tokens/s", "cores": 1, "threads": 1, "kind": "oracle",
           "sample": f"first {args.cpu_docs} docs of the same corpus ({p.T} tokens, V={p.V}), "
                     f"{args.cpu_iters} iterations after 1 warm-up, single thread", **info}
    log(f"[cpu] nytimes-shape sample {rate / 1e6:.2f}M tokens/s ({dt:.1f}s)")
    per = {}
    wl0 = synth.WORKLOADS["tiny-lda-k16"]
    c0 = wl0.make()
    r, dt = oracle_rate(c0, wl0, wl0.M, wl0.iters, 0)
    per["tiny-lda-k16"] = {"tokens_per_s": r, "sample": f"whole corpus ({c0.T} tokens), "
                           f"{wl0.iters} iterations after init", "seconds": dt}
    for name, docs in (("pubmed-shape-k1e4", 200_000), ("clueweb-share-k1e6", 120_000)):
        wl = synth.WORKLOADS[name]
        cs = wl.make(docs)
        r, dt = oracle_rate(cs, wl, wl.M, 1, 0)
        per[name] = {"tokens_per_s": r, "sample": f"first {docs} documents ({cs.T} tokens), "
                     f"1 iteration after init", "seconds": dt}
        log(f"[cpu] {name} sample {r / 1e6:.2f}M tokens/s ({dt:.1f}s)")
        del cs
    out["per_workload"] = per
    return out


def measure(W, c, wl, M, steps, warmup, dev, tag, word_alias=False):
    """Throughput of `steps` iterations after `warmup`, with the per-kernel
    times (HIP events around every launch on the sampler's stream), the
    roofline of the kernel that takes the most time and of the whole sweep.
    word_alias: word proposals of words with L_w > K from alias tables."""
    import torch
    t0 = time.perf_counter()
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, wl.K, M, wl.alpha, wl.beta, seed=1, device=dev,
                  word_alias=word_alias)
    s.init()
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    s.iterate(warmup)
    torch.cuda.synchronize()
    s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = s.profile_read()
    s.profile(False)
    kernels = {}
    for name, (launches, tokens, total_ms) in stats.items():
        if launches == 0 or tokens == 0:
            continue
        avg = total_ms / launches
        bpt = algorithmic_bytes_per_token(name, M)
        kernels[name] = dict(avg_ms=avg, tokens=tokens, gbps=bpt * tokens / (avg * 1e-3) / 1e9)
        log(f"[{tag}]   {name:16s} {avg:8.4f} ms/launch  {tokens:>11d} tokens  "
            f"{kernels[name]['gbps']:8.1f} GB/s algorithmic")
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    iter_bytes = (20 + 16 * M) * c.T
    sweep_gbps = iter_bytes * steps / dt / 1e9
    ll = s.log_likelihood()
    s.close()
    del s
    torch.cuda.empty_cache()
    log(f"[{tag}] T={c.T} K={wl.K} M={M}: {dt * 1e3 / steps:.3f} ms/iteration, "
        f"{c.T * steps / dt / 1e9:.2f}G tokens/s, sweep {sweep_gbps:.0f} GB/s algorithmic, "
        f"dominant {dom} {kernels[dom]['gbps']:.0f} GB/s, LL {ll:.6e} (create+init {t_create:.1f}s)")
    return {
        "tokens_per_s": c.T * steps / dt, "ms_per_step": dt * 1e3 / steps, "steps": steps,
        "warmup": warmup, "tokens": c.T, "V": c.V, "D": c.D, "K": wl.K, "M": M,
        "alpha": wl.alpha, "beta": wl.beta,
        "sweep": {"algorithmic_bytes_per_token": 20 + 16 * M, "gbps": sweep_gbps,
                  "frac": sweep_gbps / HBM_PEAK_GBS},
        "dominant": {"kernel": dom, "avg_ms": kernels[dom]["avg_ms"], "gbps": kernels[dom]["gbps"],
                     "frac": kernels[dom]["gbps"] / HBM_PEAK_GBS},
        "kernels_ms": {k: round(v["avg_ms"], 4) for k, v in kernels.items()},
        "log_likelihood": ll,
    }


# --------------------------------------------------------------------------
# Learned proposal + serving (fold-in of new documents against the fit)
# --------------------------------------------------------------------------
SWEEP_GRID = [1, 2, 3, 4, 5, 6, 8, 10, 12, 14, 16, 20, 24, 28, 32, 36, 40, 48, 56, 64, 80, 96, 128, 160, 200]


def corpus_features(W, c, buckets, dev):
    """CSR encoder inputs of every document of a corpus, on the device."""
    import numpy as np
    import torch
    counts = np.bincount(c.doc_ids, minlength=c.D)
    docptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint64)
    order = np.argsort(c.doc_ids, kind="stable")
    rowptr, idx, val = W.features_csr(buckets, docptr, c.word_ids[order])
    return (torch.from_numpy(rowptr.astype(np.int32)).to(dev),
            torch.from_numpy(idx.astype(np.int32)).to(dev), torch.from_numpy(val).to(dev))


def train_encoder(W, s, c, wl, dev, epochs, batch, hidden=512, buckets=100_000, lr=2e-3,
                  w1_std=1.0, n_val=8192, avg_iters=20):
    """Adam on the sampler's own (document, theta_hat_d) pairs, theta_hat_d
    averaged over the sampler's next avg_iters iterations (one state of the
    chain is a noisy target); the last n_val documents are held out to report
    the KL gap to their targets."""
    import torch
    import synth
    t0 = time.perf_counter()
    d_rp, d_idx, d_val = corpus_features(W, c, buckets, dev)
    theta = torch.zeros((c.D, wl.K), dtype=torch.float32, device=dev)
    for _ in range(avg_iters):
        s.iterate(1)
        theta += s.theta(0, c.D)
    theta /= avg_iters
    enc = W.Encoder(buckets, hidden, wl.K, max_batch=batch, lr=lr, device=dev)
    enc.set_weights(synth.encoder_init_weights(buckets, hidden, wl.K, 11, w1_std))
    n_train = c.D - n_val

    def val_loss():
        tot = 0.0
        for b0 in range(n_train, c.D, batch):
            b1 = min(c.D, b0 + batch)
            q = enc.forward(d_rp[b0:b1 + 1], d_idx, d_val).clamp_min(1e-30)
            tot += float(-(theta[b0:b1] * q.log()).sum())
        return tot / n_val

    th = theta[n_train:].double()
    ent = float(-(th * th.log()).sum(1).mean())     # floor of the soft cross-entropy
    v0 = val_loss()
    t_feat = time.perf_counter() - t0
    t1 = time.perf_counter()
    steps, curve = 0, []
    for ep in range(epochs):
        for b0 in range(0, n_train - batch + 1, batch):
            enc.train_step(d_rp[b0:b0 + batch + 1], d_idx, d_val, theta[b0:b0 + batch], want_loss=False)
            steps += 1
        if ep % 4 == 3 or ep == epochs - 1:
            curve.append((ep + 1, val_loss()))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    v1 = curve[-1][1]
    log(f"[serve] encoder: features {t_feat:.1f}s, {steps} steps in {t_train:.1f}s, held-out "
        f"loss {v0:.4f} -> {v1:.4f}, target entropy {ent:.4f}: KL {v0 - ent:.4f} -> {v1 - ent:.4f}")
    del theta, d_rp, d_idx, d_val
    return enc, dict(steps=steps, train_s=t_train, epochs=epochs, batch=batch, hidden=hidden,
                     buckets=buckets, lr=lr, target_average_iterations=avg_iters, heldout_docs=n_val, heldout_loss_first=v0,
                     heldout_loss_last=v1, target_entropy=ent, heldout_kl_first=v0 - ent,
                     heldout_kl_last=v1 - ent, kl_gap_closed=1.0 - (v1 - ent) / (v0 - ent),
                     heldout_loss_by_epoch=curve)


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
    """Smallest S on the grid from which the held-out LL stays within tol
    (relative) of ref_ll."""
    ok = [abs(curve[S] - ref_ll) <= tol * abs(ref_ll) for S in SWEEP_GRID]
    for i, S in enumerate(SWEEP_GRID):
        if all(ok[i:]):
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


def serving_experiment(W, dev, args, workload="nytimes-shape-lda-k1e3"):
    """Learned vs plain fold-in against a model frozen from a K=1000 fit.

    The fit runs on an LDA-generated NYTimes-shaped corpus with sparse topics
    (an iid-Zipf corpus has no topics to fold in against).  New documents are
    drawn from the fitted model and split 50/50 into observed and held-out
    tokens.  S* is the fewest sweeps from which the held-out LL stays within
    1% (and 0.1%) of a 200-sweep plain chain; the server then runs Poisson
    arrivals at each chain's S* (1%)."""
    import numpy as np
    import torch
    import synth
    t0 = time.perf_counter()
    wl = synth.WORKLOADS[workload]
    c = wl.make()
    log(f"[serve] {workload}: T={c.T} generated in {time.perf_counter() - t0:.1f}s")
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, wl.K, wl.M, wl.alpha, wl.beta, seed=1,
                  device=dev)
    s.init()
    s.iterate(args.fit_iters)
    torch.cuda.synchronize()
    fit_ll = s.log_likelihood()
    log(f"[serve] fit {args.fit_iters} iterations, LL {fit_ll:.6e} ({time.perf_counter() - t0:.1f}s)")
    z, _ = s.assignments()
    gm = W.Model(c.word_ids, c.doc_ids, z, c.V, c.D, wl.K, s.M, wl.alpha, wl.beta, seed=5,
                 device=dev)
    enc, enc_stats = train_encoder(W, s, c, wl, dev, args.enc_epochs, args.enc_batch)
    s.close()
    ev = synth.docs_from_model(c.word_ids, z, c.V, wl.K, 0.01, wl.beta, args.serve_eval, 31)
    rq = synth.docs_from_model(c.word_ids, z, c.V, wl.K, 0.01, wl.beta, args.serve_requests, 32)
    del z
    req = np.arange(args.serve_eval, dtype=np.uint32)
    ls = args.learned_steps
    c_plain = foldin_curve(gm, ev[0], ev[1], req, ev[2], ev[3])
    ref = c_plain[200]
    w_ev = encoder_weights(W, enc, ev[0], ev[1], dev)
    c_learn = foldin_curve(gm, ev[0], ev[1], req, ev[2], ev[3], w_ev, ls)
    # ablation: the same chain with an untrained encoder's proposal
    enc0 = W.Encoder(enc.buckets, enc.hidden, wl.K, max_batch=enc.max_batch, device=dev)
    enc0.set_weights(synth.encoder_init_weights(enc.buckets, enc.hidden, wl.K, 11, 1.0))
    c_rand = foldin_curve(gm, ev[0], ev[1], req, ev[2], ev[3], encoder_weights(W, enc0, ev[0], ev[1], dev), ls)
    enc0.close()
    star = {f"{tol:g}": {"plain": sweeps_to(c_plain, ref, tol),
                         "learned": sweeps_to(c_learn, ref, tol),
                         "untrained_encoder": sweeps_to(c_rand, ref, tol)} for tol in (0.01, 0.001)}
    gap1 = (ref - c_plain[1]) / abs(ref)
    log(f"[serve] reference LL (200 plain sweeps) {ref:.1f}, plain 1-sweep gap {gap1:.4f}; "
        f"sweeps to target: {star}")
    log(f"[serve] plain curve   {c_plain}")
    log(f"[serve] learned curve {c_learn}")
    log(f"[serve] untrained-encoder curve {c_rand}")
    arrivals = synth.poisson_arrivals(args.serve_requests, args.serve_rate, 33)
    res = {"workload": workload, "fit_iterations": args.fit_iters, "fit_ll": fit_ll,
           "reference_ll_200_plain": ref, "plain_1_sweep_gap": gap1, "eval_docs": args.serve_eval,
           "requests": args.serve_requests, "arrival_rate_per_s": args.serve_rate,
           "learned_steps": ls, "encoder": enc_stats, "sweeps_to_target": star,
           "curve_plain": c_plain, "curve_learned": c_learn, "curve_untrained_encoder": c_rand}
    sp, sl = star["0.01"]["plain"], star["0.01"]["learned"]
    if sp is not None:
        res["plain"] = serve(W, gm, None, rq[0], rq[1], rq[2], rq[3], arrivals, sp)
        log(f"[serve] plain   {res['plain']}")
    if sl is not None:
        res["learned"] = serve(W, gm, enc, rq[0], rq[1], rq[2], rq[3], arrivals, sl, ls=ls)
        log(f"[serve] learned {res['learned']}")
    if sp is not None and sl is not None:
        res["target_1pct_met"] = bool(sl < sp and res["learned"]["p99_ms"] < res["plain"]["p99_ms"])
    res["total_s"] = time.perf_counter() - t0
    enc.close()
    gm.close()
    return res


# Other single-GPU workloads measured beside the headline: (key, workload,
# M, documents or None for all).  The ClueWeb-shaped share is measured on its
# first 2M documents (about 200M tokens; its head word has ~25M tokens, far
# more than K, so the inverse-CDF path for long columns is timed).
EXTRA = [("pubmed-shape-k1e4", "pubmed-shape-k1e4", 4, None),
         ("pubmed-shape-k1e4-m2", "pubmed-shape-k1e4", 2, None),
         ("clueweb-share-k1e6-2m-docs", "clueweb-share-k1e6", 2, 2_000_000)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="nytimes-shape-k1e3")
    ap.add_argument("--M", type=int, default=None, help="override the MH steps")
    ap.add_argument("--extra-steps", type=int, default=3)
    ap.add_argument("--no-extra-configs", action="store_true",
                    help="measure the headline workload only")
    ap.add_argument("--cpu-docs", type=int, default=30000)
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the learned-proposal fold-in / serving measurement")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-eval", type=int, default=1000)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--fit-iters", type=int, default=1000,
                    help="iterations of the fit that the fold-in model is frozen from")
    ap.add_argument("--enc-epochs", type=int, default=8)
    ap.add_argument("--learned-steps", type=int, default=1,
                    help="MH steps per token and sweep with the learned proposal")
    ap.add_argument("--enc-batch", type=int, default=512)
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

    head = measure(W, c, wl, M, args.steps, args.warmup, dev, "bench")
    dom = head["dominant"]
    out = {
        "metric": "sampled tokens/s/GPU",
        "value": head["tokens_per_s"],
        "unit": "tokens/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "tokens": c.T, "V": c.V, "D": c.D, "K": wl.K,
                   "M": M, "alpha": wl.alpha, "beta": wl.beta, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom["kernel"], "achieved": dom["gbps"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["frac"],
                     "traffic": measured_traffic(args.workload, dom["kernel"]),
                     "sweep_achieved": head["sweep"]["gbps"], "sweep_frac": head["sweep"]["frac"]},
        "kernels_ms": head["kernels_ms"],
    }
    if not args.no_extra_configs:
        configs = {}
        for key, name, m, docs in EXTRA:
            if name == args.workload and m == M and docs is None:
                continue
            ewl = synth.WORKLOADS[name]
            t0 = time.perf_counter()
            ec = ewl.make(docs) if docs is not None else ewl.make()
            log(f"[bench] corpus {key}: T={ec.T} ({time.perf_counter() - t0:.1f}s)")
            r = measure(W, ec, ewl, m, args.extra_steps, 1, dev, key)
            r["workload"] = name
            if docs is not None:
                r["documents"] = f"first {docs} of {name}"
                r["longest_column"] = int(np.bincount(ec.word_ids).max())
            r["traffic"] = measured_traffic(key, r["dominant"]["kernel"])
            configs[key] = r
            del ec
        # the same workload with Walker's alias tables for the words with
        # L_w > K (all of them on the long-word kernels) instead of the
        # inverse CDF: the cost of the paper's own word proposal
        r = measure(W, c, wl, M, args.extra_steps, 1, dev, "alias", word_alias=True)
        r["workload"] = args.workload
        r["word_proposal"] = "alias table (words with L_w > K)"
        configs[args.workload + "-word-alias"] = r
        out["configs"] = configs
    if not args.no_serving:
        out["serving"] = serving_experiment(W, dev, args)
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(c, args)
        log(f"[bench] cpu baselines {time.perf_counter() - t0:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
