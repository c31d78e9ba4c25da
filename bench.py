"""Benchmark of the set-to-set scoring path on one MI355X.

Default workload: exhaustive exact-vs-BF16 scoring of 1,000 query sets (32
vectors each) against a 100,000-document corpus (lognormal set lengths, mean 80,
clipped to 32..256, ~8.0M vectors, d = 128; seeded synthetic Gaussian-mixture
embeddings standing in for the paper's ColBERT corpora). One step is the whole
exact path for the batch: query conversion to bf16, the MFMA scoring of every
(query, document) pair (dot products, per-document max, per-query sum) and the
per-query top-100. The corpus conversion (f32 -> bf16 / FP8) happens once,
before the timed region, and is reported separately.

Reported beside the step: the float32 exact path on the same batch, the FP8
estimate -> top-1000 shortlist -> float32 rerank -> top-100 path with its
recall@100 against float64 exact scores, the dominant kernel's roofline
figures, and the CPU oracle timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload {2,4,5}]
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_2603_20336_amd as gem  # noqa: E402
from paper_2603_20336_amd import workloads as wl  # noqa: E402

PEAK_BF16 = 2.5e15
PEAK_FP8 = 5.0e15
PEAK_FP4 = 10.1e15
PEAK_FP6 = 10.1e15
PEAK_FP32_MATRIX = 157.3e12
PEAK_HBM = 8.0e12


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed(fn, reps: int, stream=None):
    """Mean milliseconds of fn() over reps, from HIP events on the current stream."""
    s = torch.cuda.current_stream() if stream is None else stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def timed_once(fn, stream=None):
    """(milliseconds, result) of one call of fn(), from HIP events on the current stream."""
    s = torch.cuda.current_stream() if stream is None else stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    out = fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1), out


def build_codebook(D32, n_iter: int, assign: str, seed: int, per_centroid: int = 64):
    """C_quant for a corpus: k-means (Lloyd, n_iter rounds) on a seeded sample of
    per_centroid rows per centroid, from seeded initial rows; then every corpus
    vector's code. Returns (codebook, code sets, timings)."""
    dev = D32.device
    V = D32.n_vecs
    k1 = gem.codebook_size(V)
    n_sample = min(V, per_centroid * k1)
    rng = np.random.default_rng(seed)
    rows = torch.from_numpy(np.sort(rng.choice(V, n_sample, replace=False)).astype(np.int64)).to(dev)
    xs = torch.empty(n_sample, 128, dtype=torch.float32, device=dev)
    gem.copy_rows(D32.vecs, xs, src_idx=rows)
    init = torch.from_numpy(rng.choice(n_sample, k1, replace=False).astype(np.int64))
    t_km, C = timed_once(lambda: gem.kmeans(xs, init, n_iter, assign=assign))
    del xs
    t_enc, Dc = timed_once(lambda: gem.encode(D32, C, assign=assign))
    info = {"codebook_size": k1, "kmeans_sample_rows": n_sample, "kmeans_iters": n_iter, "assign": assign,
            "kmeans_ms": t_km, "encode_corpus_ms": t_enc,
            "encode_tflops": 2.0 * 128 * V * k1 / (t_enc / 1e3) / 1e12}
    return C, Dc, info


def bench_graph_search(seed: int = 13):
    """Alg. 5 on a kNN graph of the topical 100k corpus: C_quant (k-means of the
    vectors), C_index (k-means of the C_quant centroids) and the TF-IDF set
    clusters (Sec. 4.1), the C Q^T filter, and the batched search of all
    queries with the FP8 estimate, then the exact f32 rerank of R; recall
    against the exhaustive float32 top-k."""
    from paper_2603_20336_amd import search as gs
    dev = torch.device("cuda:0")
    w6 = wl.WORKLOADS[6]
    k = w6.k
    log("graph search: topical 100k corpus")
    c, q = wl.corpus(w6, device=dev), wl.queries(w6, device=dev)
    D32 = gem.Sets(c.vecs, c.offsets, "f32", c.max_len())
    Q = gem.Sets(q.vecs, q.offsets, "f32", q.max_len())
    D8 = gem.quantize_fp8(D32)
    C_quant, Dc, cb = build_codebook(D32, n_iter=8, assign="f32", seed=seed)
    _, exact_ids = gem.score_exact(Q, D32, compute="f32", k=k)
    t_exh = timed(lambda: gem.score_exact(Q, D32, cands=gem.Cands(gem.topk(gem.score_quant(gem.quantize_fp8(Q), D8),
                                                                           1000)[1].reshape(-1), stride=1000,
                                                                  n_lists=Q.n_sets), compute="f32", k=k), 1)
    res = {"workload": w6.name, "docs": D32.n_sets, "doc_vectors": D32.n_vecs, "queries": Q.n_sets, "k": k,
           "codebook_size": cb["codebook_size"], "exhaustive_fp8_rerank_ms": t_exh}
    k2, r, t, degree, width = 128, 2, 4, 24, 4
    rng = np.random.default_rng(seed)
    init = torch.from_numpy(rng.choice(C_quant.shape[0], k2, replace=False).astype(np.int64))
    t_idx, C_index = timed_once(lambda: gem.kmeans(C_quant, init, 6))
    vc = gem.nearest_centroid(D32.vecs, C_index)
    masks, moff, members = gs.set_clusters(vc, D32.offsets, k2, r)
    torch.cuda.synchronize()
    t_graph, nbrs = timed_once(lambda: gs.knn_graph(D32, D8, degree, batch=2000))
    index = gs.ClusterIndex(nbrs, masks, moff, members, C_index)
    res.update({"k2": k2, "r": r, "t": t, "degree": degree, "width": width, "index_kmeans_ms": t_idx,
                "knn_graph_ms": t_graph, "mean_clusters_per_set": float(moff[-1].item()) / D32.n_sets})
    Q8 = gem.quantize_fp8(Q)
    n_q = Q.n_sets
    words = torch.from_numpy(rng.integers(0, 2 ** 32, (n_q, k2), dtype=np.uint64).astype(np.uint32).view(np.int32))
    words = words.to(dev)
    runs = []
    for ef in (32, 64, 128, 256):
        def go(ef=ef):
            qmask = gs.query_clusters(Q, C_index, t)
            srch = gs.GraphSearch(Q8, D8, index, qmask, ef=ef, width=width)
            srch.run(words, check_every=4)                      # 4 steps per graph replay
            return srch, srch.rerank(Q, D32, k)
        go()                                                     # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        srch, (_, top) = go()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        vis = srch.visited.view(torch.uint8)
        scored = torch.stack([(vis >> b) & 1 for b in range(8)]).sum().item() / n_q
        tn, en = top.cpu().numpy(), exact_ids.cpu().numpy()
        rec = float(np.mean([len(set(tn[i][:k]) & set(en[i][:k])) / k for i in range(n_q)]))
        # of the exact top-k: the share the search scored at all, and the share in R
        ex = exact_ids.long()
        vbits = (srch.visited.gather(1, (ex >> 5)) >> (ex & 31)) & 1
        reached = float(vbits.float().mean().item())
        bi = srch.beam.ids.cpu().numpy()
        in_r = float(np.mean([len(set(bi[i]) & set(en[i][:k])) / k for i in range(n_q)]))
        runs.append({"ef": ef, "ms": ms, "qps": n_q / (ms / 1e3), "steps": srch.steps,
                     "sets_scored_per_query": scored, f"recall_at_{k}_vs_f32_exact": rec,
                     "exact_topk_scored": reached, "exact_topk_in_R": in_r})
        log(f"graph search ef={ef}: {ms:.1f} ms for {n_q} queries, {srch.steps} steps, "
            f"{scored:.0f} sets scored per query, recall@{k} {rec:.3f} (exact top-{k}: {reached:.3f} scored, "
            f"{in_r:.3f} in R)")
    res["runs"] = runs
    # what bounds the recall: the share of the exact top-k that passes the
    # cluster test, and the same search without it
    qmask = gs.query_clusters(Q, C_index, t)
    pm = masks[exact_ids.long()]                                    # [n_q, k, words]
    res["exact_topk_passing_cluster_filter"] = float(((pm & qmask[:, None, :]) != 0).any(-1).float().mean().item())
    srch = gs.GraphSearch(Q8, D8, index, torch.full_like(qmask, -1), ef=128, width=width)
    srch.run(words, check_every=4)
    _, top = srch.rerank(Q, D32, k)
    tn, en = top.cpu().numpy(), exact_ids.cpu().numpy()
    res["recall_without_cluster_filter_ef128"] = float(np.mean([len(set(tn[i][:k]) & set(en[i][:k])) / k
                                                              for i in range(n_q)]))
    log(f"exact top-{k} passing the cluster filter: {res['exact_topk_passing_cluster_filter']:.3f}; "
        f"recall without the filter (ef 128): {res['recall_without_cluster_filter_ef128']:.3f}")
    # EMD of graph edges (Sec. 4.2: the construction metric), on the vectors and
    # as qEMD on the codes; entropic, eps 0.05, 50 Sinkhorn rounds
    n_pairs = 20000
    a_idx = torch.from_numpy(rng.integers(0, D32.n_sets, n_pairs).astype(np.int32)).to(dev)
    b_idx = nbrs[a_idx.long(), 1].contiguous()
    emd = {"pairs": n_pairs, "eps": 0.05, "n_iter": 50}
    for name, S in (("emd_vectors", D32), ("qemd_codes", Dc)):
        gem.emd_sinkhorn(S, S, a_idx[:64], b_idx[:64], 0.05, 50)
        ms = timed(lambda S=S: gem.emd_sinkhorn(S, S, a_idx, b_idx, 0.05, 50), 1)
        emd[name] = {"ms": ms, "pairs_per_s": n_pairs / (ms / 1e3)}
        log(f"{name}: {n_pairs} pairs in {ms:.1f} ms")
    res["emd_sinkhorn"] = emd
    return res


def host_cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(q: wl.SetBatch, c: wl.SetBatch, n_sample: int):
    """The float64 oracle on a bounded sample of queries against the whole corpus."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    sub = q.subset(list(range(n_sample)))
    qv, qo = sub.vecs.numpy(), sub.offsets.numpy()
    dv, do = c.vecs.numpy(), c.offsets.numpy()
    t0 = time.perf_counter()
    ref = oracle.ch_dense(qv, qo, dv, do)
    dt = time.perf_counter() - t0
    return ref, {"value": n_sample * c.n_sets / dt, "unit": "pair-scores/s", "cores": int(cores),
                 "cpu_model": host_cpu_model(), "host_cpus": os.cpu_count(),
                 "kind": "oracle",
                 "sample": f"{n_sample} query sets x {c.n_sets} documents, float64 NumPy/BLAS, {dt:.1f} s"}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "score_dense_bf16_exhaustive100k_traffic.txt")
DENSE_SOURCES = [os.path.join(ROOT, "paper_2603_20336_amd", "csrc", f)
                 for f in ("score.hip", "mfma_ops.hpp", "device_common.hpp", "gem_internal.h")]


def dense_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in DENSE_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dense bf16 kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by the copy-kernel factor);
    None when there is none or the kernel's sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith("#"))
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        if kv.get("source_sha256") != dense_source_digest():
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def copy_calibration(n_bytes: int = 1 << 30, reps: int = 3) -> None:
    """A plain streaming copy of known size (read n_bytes, write n_bytes), run
    for the counter runs that scale FETCH_SIZE / WRITE_SIZE to bytes."""
    src = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log(f"copy calibration: {reps} x {n_bytes} bytes read + written")


def recall_gpu(top_ids: torch.Tensor, exact: torch.Tensor, exact_kth: torch.Tensor, k: int) -> float:
    """Recall@k (Sec. 5.1) of every query's returned ids against its exact
    float32 scores, tie-aware: a returned id counts when its exact score is at
    least the exact k-th score minus a band of 2e-4 * max(|s_k|, 1)."""
    ids = top_ids[:, :k].long()
    valid = ids >= 0
    s = exact.gather(1, ids.clamp(min=0))
    tau = 2e-4 * exact_kth.abs().clamp(min=1.0)
    hits = ((s >= (exact_kth - tau)[:, None]) & valid).float().sum(1)
    return float((hits / k).mean().item())


def bench_exhaustive(args):
    import oracle
    dev = torch.device("cuda:0")
    w2 = wl.WORKLOADS[2]
    log("generating the 100k-document corpus and 1000 queries on the GPU")
    c_dev = wl.corpus(w2, device=dev)
    q_dev = wl.queries(w2, device=dev)
    n_q, n_d = q_dev.n_sets, c_dev.n_sets
    V = c_dev.n_vecs
    q_rows = q_dev.n_vecs
    log(f"corpus: {n_d} sets, {V} vectors; queries: {n_q} sets, {q_rows} vectors")

    Q = gem.Sets(q_dev.vecs, q_dev.offsets, "f32", q_dev.max_len())
    D32 = gem.Sets(c_dev.vecs, c_dev.offsets, "f32", c_dev.max_len())

    # a1: corpus conversion, once (timed on its own)
    torch.cuda.synchronize()
    t_bf16 = timed(lambda: gem.convert_bf16(D32), 1)
    t_fp8 = timed(lambda: gem.quantize_fp8(D32), 1)
    D16 = gem.convert_bf16(D32)
    D8 = gem.quantize_fp8(D32)
    torch.cuda.synchronize()

    k = w2.k
    flops = 2.0 * 128 * q_rows * V
    pairs = n_q * n_d
    scores = torch.empty(n_q, n_d, dtype=torch.float32, device=dev)
    # the autotuner picks the dense scorer's schedule for this shape (untimed)
    sched = {}
    sched["bf16"], _ = gem.autotune_dense(gem.convert_bf16(Q), D16, reps=2, scores=scores)
    log(f"bf16 schedule {sched['bf16']}")
    ws_fused = gem.score_workspace_bytes(Q, D16, k=k, compute="bf16")

    def step():
        Q16 = gem.convert_bf16(Q)                                   # a2: query ingest
        return gem.score_exact(Q16, D16, compute="bf16", k=k)       # a3-a6: MFMA scoring, fused top-100

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # per-stage timings (events on the stream the kernels run on)
    Q16 = gem.convert_bf16(Q)
    t_conv = timed(lambda: gem.convert_bf16(Q), max(1, args.steps))
    t_fused = timed(lambda: gem.score_exact(Q16, D16, compute="bf16", k=k), max(1, args.steps))
    t_score = timed(lambda: gem.score_exact(Q16, D16, compute="bf16", scores=scores), max(1, args.steps))
    t_topk = timed(lambda: gem.topk(scores, k), max(1, args.steps))
    gem.set_topk_fusion("staged")
    ws_staged = gem.score_workspace_bytes(Q, D16, k=k, compute="bf16")
    gem.set_topk_fusion("auto")

    torch.cuda.synchronize()
    gc.disable()                        # no collector pause inside the timed steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        top_s, top_i = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gc.enable()
    ms_per_step = dt * 1e3 / args.steps
    log(f"bf16 step {ms_per_step:.2f} ms (convert {t_conv:.3f}, fused score+top-{k} {t_fused:.2f}; "
        f"staged: score {t_score:.2f} + top-k {t_topk:.2f})")
    bf16_sample = scores[:max(1, args.cpu_sample)].clone()     # the bf16 scores of the accuracy sample

    # float32 exact path (the "plain FP32 GPU path") on the same batch; its
    # full score rows are the reference every recall below is taken against
    sched["f32"], _ = gem.autotune_dense(Q, D32, reps=1, scores=scores)
    exact = torch.empty(n_q, n_d, dtype=torch.float32, device=dev)
    gem.score_exact(Q, D32, compute="f32", scores=exact)
    top32_s, top32_i = gem.topk(exact, k)
    torch.cuda.synchronize()
    t_f32 = timed(lambda: gem.score_exact(Q, D32, compute="f32", k=k), 1)
    exact_kth = top32_s[:, k - 1].clone()
    log(f"f32 exact path {t_f32:.1f} ms")

    # the exact mode that takes each float32 product as three bfloat16
    # products (corpus split once, queries split in the workspace)
    t_split = timed(lambda: gem.split_bf16x3(D32), 1)
    Dx3 = gem.split_bf16x3(D32)
    sched["bf16x3"], _ = gem.autotune_dense(Q, Dx3, reps=1, scores=scores)
    x3_s, x3_i = gem.score_exact(Q, Dx3, compute="bf16x3", k=k)
    torch.cuda.synchronize()
    t_x3 = timed(lambda: gem.score_exact(Q, Dx3, compute="bf16x3", k=k), max(1, args.steps // 4))
    gem.score_exact(Q, Dx3, compute="bf16x3", scores=scores)
    x3_sample = scores[:max(1, args.cpu_sample)].clone()
    log(f"bf16x3 exact path {t_x3:.1f} ms ({t_f32 / t_x3:.2f}x the f32 path)")

    def rerank(short_i, sl):
        C = gem.Cands(short_i.reshape(-1), stride=sl, n_lists=n_q)
        return gem.score_exact(Q, D32, cands=C, compute="f32", k=k)

    def rerank_x3(short_i, sl):
        # the exact rerank in split-bf16 products (within the exactness bound)
        C = gem.Cands(short_i.reshape(-1), stride=sl, n_lists=n_q)
        return gem.score_exact(Q, Dx3, cands=C, compute="bf16x3", k=k)

    # estimate -> top-sl shortlist -> float32 rerank -> top-100, swept over
    # the shortlist length (Sec. 5, "Effect of #rerank")
    sweep_sl = [int(x) for x in args.shortlists.split(",") if x]

    def sweep(name, make_q, score_k, rr=rerank):
        out = {}
        for sl in sweep_sl:
            def path(sl=sl):
                _, short_i = score_k(make_q(), sl)
                return rr(short_i, sl)
            r_s, r_i = path()
            torch.cuda.synchronize()
            t = timed(path, max(1, args.steps // 4))
            out[str(sl)] = {"ms": t, "pair_scores_per_s": pairs / (t / 1e3), "speedup_vs_f32_path": t_f32 / t,
                            f"recall_at_{k}": recall_gpu(r_i, exact, exact_kth, k)}
            log(f"{name} shortlist {sl}: {t:.2f} ms, recall@{k} {out[str(sl)][f'recall_at_{k}']:.4f}")
        return out, r_s, r_i

    # FP8 E4M3 estimate
    Q8 = gem.quantize_fp8(Q)
    est = torch.empty(n_q, n_d, dtype=torch.float32, device=dev)
    sched["fp8"], _ = gem.autotune_dense(Q8, D8, reps=2, scores=est)
    t_fp8_score = timed(lambda: gem.score_quant(Q8, D8, scores=est), max(1, args.steps))
    fp8_sample = est[:max(1, args.cpu_sample)].clone()
    fp8_sweep, r8_s, r8_i = sweep("fp8", lambda: gem.quantize_fp8(Q), lambda q8, sl: gem.score_quant(q8, D8, k=sl))
    fp8_x3_sweep, _, _ = sweep("fp8 -> split-bf16 rerank", lambda: gem.quantize_fp8(Q),
                               lambda q8, sl: gem.score_quant(q8, D8, k=sl), rr=rerank_x3)
    r8_s, r8_i = rerank(gem.score_quant(gem.quantize_fp8(Q), D8, k=1000)[1], 1000)

    # the rerank of the FP8 top-1000 (1M entries over about 26k distinct
    # documents) by query, by document and in the mixed order (auto), in
    # float32 and in split-bf16
    short1000 = gem.score_quant(gem.quantize_fp8(Q), D8, k=1000)[1]
    C1000 = gem.Cands(short1000.reshape(-1), stride=1000, n_lists=n_q)
    rerank_orders = {"entries": n_q * 1000, "distinct_docs": int(torch.unique(short1000).numel())}
    for order in ("query", "document", "auto"):
        gem.set_gather_order(order)
        rerank_orders[f"f32_by_{order}_ms"] = timed(
            lambda: gem.score_exact(Q, D32, cands=C1000, compute="f32", k=k), max(1, args.steps // 4))
        rerank_orders[f"bf16x3_by_{order}_ms"] = timed(
            lambda: gem.score_exact(Q, Dx3, cands=C1000, compute="bf16x3", k=k), max(1, args.steps // 4))
    gem.set_gather_order("auto")
    _, rx3_i = gem.score_exact(Q, Dx3, cands=C1000, compute="bf16x3", k=k)
    rerank_orders[f"bf16x3_rerank_recall_at_{k}"] = recall_gpu(rx3_i, exact, exact_kth, k)
    log(f"rerank of the FP8 top-1000: {rerank_orders}")
    del Dx3, C1000, short1000

    # MXFP4 estimate (E2M1 codes, a power-of-two scale per 32 dims)
    D4 = gem.quantize_mxfp4(D32)
    Q4 = gem.quantize_mxfp4(Q)
    sched["mxfp4"], _ = gem.autotune_dense(Q4, D4, reps=2, scores=est)
    t_mx_score = timed(lambda: gem.score_quant(Q4, D4, scores=est), max(1, args.steps))
    mx_sweep, _, _ = sweep("mxfp4", lambda: gem.quantize_mxfp4(Q), lambda q4, sl: gem.score_quant(q4, D4, k=sl))
    del D4, Q4
    # MXFP6 (E2M3) estimate
    D6 = gem.quantize_mxfp6(D32)
    Q6 = gem.quantize_mxfp6(Q)
    sched["mxfp6"], _ = gem.autotune_dense(Q6, D6, reps=2, scores=est)
    t_mx6_score = timed(lambda: gem.score_quant(Q6, D6, scores=est), max(1, args.steps))
    mx6_sweep, _, _ = sweep("mxfp6", lambda: gem.quantize_mxfp6(Q), lambda q6, sl: gem.score_quant(q6, D6, k=sl))
    del D6, Q6

    # qCH (Sec. 4.5): every vector replaced by its nearest centroid of the
    # k-means codebook (Secs. 4.1, 4.2); estimate -> shortlist -> f32 rerank
    log("qCH: k-means codebook and corpus codes")
    C, Dc, qch = build_codebook(D32, n_iter=8, assign="f32", seed=7)
    for cdt in ("bf16", "fp8"):
        Dcc = Dc.to_bf16() if cdt == "bf16" else Dc.to_fp8()

        def make_qc(cdt=cdt):
            Qc = gem.encode(Q, C, assign="f32")                        # NN(q) of every query vector
            return Qc.to_bf16() if cdt == "bf16" else Qc.to_fp8()

        def score_k(Qcc, sl, cdt=cdt, Dcc=Dcc):
            if cdt == "bf16":
                return gem.score_exact(Qcc, Dcc, compute="bf16", k=sl)
            return gem.score_quant(Qcc, Dcc, k=sl)

        Qcc = make_qc()
        if cdt == "bf16":
            t_sc = timed(lambda: gem.score_exact(Qcc, Dcc, compute="bf16", scores=est), max(1, args.steps // 2))
        else:
            t_sc = timed(lambda: gem.score_quant(Qcc, Dcc, scores=est), max(1, args.steps // 2))
        t_enc_q = timed(lambda: gem.encode(Q, C, assign="f32"), max(1, args.steps // 2))
        sw, _, _ = sweep(f"qCH {cdt}", make_qc, score_k)
        peak = PEAK_BF16 if cdt == "bf16" else PEAK_FP8
        qch[cdt] = {"query_encode_ms": t_enc_q, "score_ms": t_sc, "score_frac_of_peak": flops / (t_sc / 1e3) / peak,
                    "shortlist_sweep": sw}
    qch["corpus_code_bytes"] = D32.n_vecs * 4
    qch["codebook_bytes_bf16"] = qch["codebook_size"] * 256
    del C, Dc

    # accuracy: the f32 path against float64 (CPU oracle) on a sample, which
    # also times the oracle; recall of every path over all queries against
    # the f32 scores
    res = {}
    if not args.skip_cpu:
        c_host = wl.SetBatch(c_dev.vecs.cpu(), c_dev.offsets.cpu())
        q_host = wl.SetBatch(q_dev.vecs.cpu(), q_dev.offsets.cpu())
        ref, cpu = cpu_baseline(q_host, c_host, args.cpu_sample)
        ns = ref.shape[0]
        res["cpu_baseline"] = cpu
        ex_np = exact[:ns].double().cpu().numpy()
        t32 = top32_i[:ns].cpu().numpy()
        matched = 0
        for r in range(ns):
            tau = 2e-4 * max(abs(np.sort(ref[r])[::-1][k - 1]), 1.0)
            matched += int(oracle.tie_aware_match(t32[r], ref[r], k, tau)[0])
        res["f32_exact_vs_float64"] = {
            "queries": ns, "top100_match_outside_ties": f"{matched}/{ns}",
            "max_rel_err_all_scores": float((np.abs(ex_np - ref) / np.maximum(np.abs(ref), 1)).max())}
        got16 = bf16_sample[:ns].double().cpu().numpy()
        res["bf16_max_rel_err"] = float((np.abs(got16 - ref) / np.maximum(np.abs(ref), 1)).max())
        got3 = x3_sample[:ns].double().cpu().numpy()
        t3 = x3_i[:ns].cpu().numpy()
        m3 = 0
        for r in range(ns):
            tau = 2e-4 * max(abs(np.sort(ref[r])[::-1][k - 1]), 1.0)
            m3 += int(oracle.tie_aware_match(t3[r], ref[r], k, tau)[0])
        res["bf16x3_exact_vs_float64"] = {
            "queries": ns, "top100_match_outside_ties": f"{m3}/{ns}",
            "max_rel_err_all_scores": float((np.abs(got3 - ref) / np.maximum(np.abs(ref), 1)).max())}
        for name, (ts_, ti_) in (("f32", (top32_s, top32_i)), ("fp8_rerank", (r8_s, r8_i))):
            ts_np, ti_np = ts_[:ns].double().cpu().numpy(), ti_[:ns].cpu().numpy()
            rr = np.take_along_axis(ref, ti_np, axis=1)
            res[f"{name}_top100_max_rel_err"] = float((np.abs(ts_np - rr) / np.maximum(np.abs(rr), 1)).max())
        est_np = fp8_sample[:ns].double().cpu().numpy()
        res["fp8_estimate_rel_err_p50"] = float(np.median(np.abs(est_np - ref) / np.maximum(np.abs(ref), 1)))
    res["recall_at_100_bf16"] = recall_gpu(top_i, exact, exact_kth, k)
    res["recall_at_100_fp8_rerank"] = fp8_sweep.get("1000", {}).get(f"recall_at_{k}")
    res["recall_at_100_mxfp4_rerank"] = mx_sweep.get("1000", {}).get(f"recall_at_{k}")
    res["recall_at_100_mxfp6_rerank"] = mx6_sweep.get("1000", {}).get(f"recall_at_{k}")
    res["recall_queries"] = n_q
    res["recall_reference"] = "float32 exact scores of every (query, document) pair, checked against float64"
    value = pairs / (ms_per_step / 1e3)
    achieved = flops / (t_fused / 1e3)
    line = {
        "metric": "query-doc set scores/sec + recall@100 vs FP64 exact; p50/p99 query latency",
        "value": value,
        "unit": "pair-scores/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "exhaustive-100k: 1000 queries x 32 vectors vs 100k docs (lognormal 32-256, "
                               f"{V} vectors), d=128, bf16 MFMA, top-100", "n_queries": n_q, "n_docs": n_d,
                   "doc_vectors": V, "query_vectors": q_rows, "k": k},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16, "traffic": measured_traffic(),
                     "kernel": "score_dense_kernel<bf16, fused top-k>", "kernel_ms": t_fused,
                     "flops_per_launch": flops, "traffic_unit": "HBM bytes per launch",
                     "algorithmic_bytes_per_launch": V * 128 * 2 + q_rows * 128 * 2 + n_q * k * 8},
        "stages_ms": {"query_convert": t_conv, "score_dense_bf16_fused_top100": t_fused,
                      "staged_score_dense_bf16": t_score, "staged_topk_100": t_topk},
        "topk_workspace_bytes": {"fused": ws_fused, "staged": ws_staged},
        "dense_schedule": sched,
        "corpus_convert_ms": {"bf16": t_bf16, "fp8": t_fp8},
        "f32_exact_path": {"ms": t_f32, "pair_scores_per_s": pairs / (t_f32 / 1e3),
                           "tflops": flops / (t_f32 / 1e3) / 1e12,
                           "frac_of_fp32_matrix_peak": flops / (t_f32 / 1e3) / PEAK_FP32_MATRIX},
        "bf16x3_exact_path": {"ms": t_x3, "pair_scores_per_s": pairs / (t_x3 / 1e3),
                              "speedup_vs_f32_path": t_f32 / t_x3, "corpus_split_ms": t_split,
                              "tflops_algorithmic": flops / (t_x3 / 1e3) / 1e12,
                              "mfma_frac_of_bf16_peak": 3 * flops / (t_x3 / 1e3) / PEAK_BF16,
                              f"recall_at_{k}_vs_f32": recall_gpu(x3_i, exact, exact_kth, k)},
        "fp8_rerank_path": dict(fp8_sweep.get("1000", {}), shortlist=1000, fp8_score_ms=t_fp8_score,
                                fp8_tflops=flops / (t_fp8_score / 1e3) / 1e12,
                                fp8_frac_of_peak=flops / (t_fp8_score / 1e3) / PEAK_FP8,
                                shortlist_sweep=fp8_sweep, rerank_gather_orders=rerank_orders),
        "fp8_bf16x3_rerank_path": dict(fp8_x3_sweep.get("1000", {}), shortlist=1000,
                                       rerank="split-bf16 exact mode (three bf16 products per float32 product)",
                                       shortlist_sweep=fp8_x3_sweep),
        "mxfp4_rerank_path": dict(mx_sweep.get("1000", {}), shortlist=1000, mxfp4_score_ms=t_mx_score,
                                  mxfp4_tflops=flops / (t_mx_score / 1e3) / 1e12,
                                  mxfp4_frac_of_peak=flops / (t_mx_score / 1e3) / PEAK_FP4,
                                  corpus_bytes=V * 68, shortlist_sweep=mx_sweep),
        "mxfp6_rerank_path": dict(mx6_sweep.get("1000", {}), shortlist=1000, mxfp6_score_ms=t_mx6_score,
                                  mxfp6_tflops=flops / (t_mx6_score / 1e3) / 1e12,
                                  mxfp6_frac_of_peak=flops / (t_mx6_score / 1e3) / PEAK_FP6,
                                  corpus_bytes=V * 100, shortlist_sweep=mx6_sweep),
        "qch_rerank_path": qch,
    }
    line.update(res)
    if "cpu_baseline" not in line:
        line["cpu_baseline"] = None
    del exact, est, scores
    return line, (D8, D32)


def bench_rerank_orders(args):
    """The rerank of the FP8 top-1000 of workload 3 (1000 queries x 1000 ids
    over the 100k corpus) in every gather order (by query: the sorted
    chunk-major walk; by document; mixed: auto), in float32 and in split bf16,
    each order's scores checked bitwise against the query order's."""
    dev = torch.device("cuda:0")
    w2 = wl.WORKLOADS[2]
    c_dev, q_dev = wl.corpus(w2, device=dev), wl.queries(w2, device=dev)
    Q = gem.Sets(q_dev.vecs, q_dev.offsets, "f32", q_dev.max_len())
    D32 = gem.Sets(c_dev.vecs, c_dev.offsets, "f32", c_dev.max_len())
    D8, Dx3 = gem.quantize_fp8(D32), gem.split_bf16x3(D32)
    short = gem.score_quant(gem.quantize_fp8(Q), D8, k=1000)[1]
    C = gem.Cands(short.reshape(-1).contiguous(), stride=1000, n_lists=Q.n_sets)
    res = {"entries": Q.n_sets * 1000, "distinct_docs": int(torch.unique(short).numel())}
    for name, fn in (("f32", lambda: gem.score_exact(Q, D32, cands=C, compute="f32")),
                     ("bf16x3", lambda: gem.score_exact(Q, Dx3, cands=C, compute="bf16x3"))):
        ref = None
        for order in ("query", "document", "auto"):
            gem.set_gather_order(order)
            out = fn()
            torch.cuda.synchronize()
            if ref is None:
                ref = out.clone()
            res[f"{name}_{order}_bitwise_as_query"] = bool(torch.equal(out.view(torch.int32), ref.view(torch.int32)))
            res[f"{name}_{order}_ms"] = timed(fn, max(1, args.steps // 4))
            log(f"rerank {name} by {order}: {res[f'{name}_{order}_ms']:.2f} ms")
        gem.set_gather_order("auto")
    return res


def bench_dense_only(args):
    """The dense scorers alone, for counter runs: the bf16 step (fused top-100,
    then staged), and FP8, MXFP4, MXFP6 and split-bf16 exact exhaustive scoring
    into a score matrix."""
    dev = torch.device("cuda:0")
    w2 = wl.WORKLOADS[2]
    c_dev, q_dev = wl.corpus(w2, device=dev), wl.queries(w2, device=dev)
    Q = gem.Sets(q_dev.vecs, q_dev.offsets, "f32", q_dev.max_len())
    D32 = gem.Sets(c_dev.vecs, c_dev.offsets, "f32", c_dev.max_len())
    D16, D8, D4, D6 = gem.convert_bf16(D32), gem.quantize_fp8(D32), gem.quantize_mxfp4(D32), gem.quantize_mxfp6(D32)
    Q16, Q8, Q4, Q6 = gem.convert_bf16(Q), gem.quantize_fp8(Q), gem.quantize_mxfp4(Q), gem.quantize_mxfp6(Q)
    Dx3 = gem.split_bf16x3(D32)
    scores = torch.empty(Q.n_sets, D32.n_sets, dtype=torch.float32, device=dev)
    flops = 2.0 * 128 * Q.n_vecs * D32.n_vecs
    out = {}
    # (the split-bf16 exact mode runs three bf16 products per float32 product:
    # its MFMA fraction counts them against the bf16 peak)
    for name, QQ, DD, peak in (("bf16", Q16, D16, PEAK_BF16), ("fp8", Q8, D8, PEAK_FP8), ("mxfp4", Q4, D4, PEAK_FP4),
                               ("mxfp6", Q6, D6, PEAK_FP6), ("bf16x3", Q, Dx3, PEAK_BF16 / 3)):
        sched, _ = gem.autotune_dense(QQ, DD, reps=2, scores=scores)
        if name == "bf16":
            t_f = timed(lambda: gem.score_exact(QQ, DD, compute="bf16", k=100), max(1, args.steps))
            out["bf16_fused_top100_ms"] = t_f
            t = timed(lambda: gem.score_exact(QQ, DD, compute="bf16", scores=scores), max(1, args.steps))
        elif name == "bf16x3":
            t = timed(lambda: gem.score_exact(QQ, DD, compute="bf16x3", scores=scores), max(1, args.steps))
        else:
            t = timed(lambda: gem.score_quant(QQ, DD, scores=scores), max(1, args.steps))
        out[name] = {"schedule": sched, "ms": t, "frac_of_peak": flops / (t / 1e3) / peak}
        log(f"dense {name}: {t:.2f} ms ({out[name]['frac_of_peak']:.3f} of peak)")
    return out


def serving_shortlist_recall(D8, D32, shortlists, n_q=1000, q_len=("uniform", 4, 64)):
    """Recall@k of the serving path (FP8 estimate -> top-s shortlist -> float32
    rerank -> top-k) against exact float32 scores, on queries of the serving
    mix, for each shortlist length s."""
    w5 = wl.WORKLOADS[5]
    k = w5.k
    q = wl.queries(w5, n_queries=n_q, query_len=q_len)
    Q32 = gem.Sets.from_batch(q, D32.device)
    Q8 = gem.quantize_fp8(Q32)
    exact = torch.empty(n_q, D32.n_sets, dtype=torch.float32, device=D32.device)
    gem.score_exact(Q32, D32, compute="f32", scores=exact)
    top_s, _ = gem.topk(exact, k)
    exact_kth = top_s[:, k - 1].clone()
    out = {}
    for sl in shortlists:
        _, short_i = gem.score_quant(Q8, D8, k=sl)
        C = gem.Cands(short_i.reshape(-1), stride=sl, n_lists=n_q)
        _, r_i = gem.score_exact(Q32, D32, cands=C, compute="f32", k=k)
        out[str(sl)] = recall_gpu(r_i, exact, exact_kth, k)
        log(f"serving mix: FP8 shortlist {sl} -> recall@{k} {out[str(sl)]:.5f}")
    return {"queries": n_q, "query_len": f"U{{{q_len[1]}..{q_len[2]}}}", f"recall_at_{k}": out}


_SERVE_TUNED = {}


def bench_serving(D8, D32, q_len=("uniform", 4, 64), rate=2000.0, n_req=1500, n_chunks=4, rate_idx=0,
                  max_resident=None, shortlist=None, chunk_work=8192):
    """Continuous-batching serving loop on the resident corpus: QPS and p50/p99
    latency. max_resident: a device-memory budget for that many requests'
    state (None: half the free device memory); the slot count stays 1024, so
    with a small budget it is the memory check that refuses requests."""
    from paper_2603_20336_amd import serve
    w5 = wl.WORKLOADS[5]
    q = wl.queries(w5, n_queries=n_req, query_len=q_len)
    arrivals = wl.poisson_arrivals(rate, n_req, rate_idx).numpy()
    off = q.offsets.numpy()
    vecs = q.vecs.numpy()
    reqs = [serve.Request(i, vecs[off[i]:off[i + 1]], float(arrivals[i])) for i in range(n_req)]
    shortlist = w5.shortlist if shortlist is None else int(shortlist)
    ex = serve.DeviceExecutor(D8, D32, n_chunks=n_chunks, max_slots=1024, shortlist=shortlist, k=w5.k)
    global _SERVE_TUNED
    work = int(chunk_work)
    if not _SERVE_TUNED.get((shortlist, n_chunks, work)):
        # schedules for the loop's launch shapes (kept in the device context
        # for every later executor): sample queries of the serving mix, drawn
        # apart from the measured requests
        tq = wl.queries(w5, n_queries=1024, query_len=q_len, seed_offset=77)
        toff, tvecs = tq.offsets.numpy(), tq.vecs.numpy()
        t0 = time.perf_counter()
        sch = ex.autotune([tvecs[toff[i]:toff[i + 1]] for i in range(tq.n_sets)], chunk_work=work)
        log(f"serving schedules tuned in {time.perf_counter() - t0:.1f} s: "
            f"{ {k: v for k, v in sch.items() if k in ('score_fp8_64', 'score_fp8_256', 'rerank_f32_32')} }")
        _SERVE_TUNED[(shortlist, n_chunks, work)] = sch
    budget = None if max_resident is None else int(max_resident) * ex.bytes_per_request
    # an iteration scores as many chunks as fit chunk_work (query vectors x chunks)
    eng = serve.ServingEngine(ex, max_slots=1024, mem_budget_bytes=budget, chunk_work=work)
    # warm-up on a few requests, then the measured run
    warm = serve.ServingEngine(ex, max_slots=1024, chunk_work=work)
    warm.run([serve.Request(-1 - i, r.vecs, r.t_arrival) for i, r in enumerate(reqs[:200])])
    torch.cuda.synchronize()
    # the loop runs with the garbage collector paused (a full collection
    # stalls the host for tens of milliseconds, which shows as a p99 spike)
    gc.collect()
    gc.disable()
    try:
        done = eng.run(reqs)
    finally:
        gc.enable()
    st = serve.latency_stats(done)
    st.update({"rate_per_s": rate, "requests": n_req, "chunks": n_chunks, "chunk_work": work,
               "iterations": eng.iteration,
               "mean_active": eng.active_sum / max(1, eng.iteration),
               "device_budget_bytes": eng.mem_budget, "bytes_per_request": ex.bytes_per_request,
               "refused_for_memory": eng.refused_for_memory,
               "shortlist": shortlist, "k": w5.k, "query_len": f"U{{{q_len[1]}..{q_len[2]}}}"})
    return st


def bench_expansion(args):
    """Batched beam expansion on the 1M-document corpus: 20 graph-captured steps."""
    from paper_2603_20336_amd.search import ExpansionGraph
    dev = torch.device("cuda:0")
    w4 = wl.WORKLOADS[4]
    n_docs = args.expand_docs
    log(f"expansion: generating {n_docs} documents")
    c = wl.corpus(w4, device=dev, n_docs=n_docs)
    q = wl.queries(w4, device=dev)
    D32 = gem.Sets(c.vecs, c.offsets, "f32", c.max_len())
    D8 = gem.quantize_fp8(D32)
    Q32 = gem.Sets(q.vecs, q.offsets, "f32", q.max_len())
    Q8 = gem.quantize_fp8(Q32)
    steps, uniq_bytes, pair_bytes = [], 0, 0
    lens = (c.offsets[1:] - c.offsets[:-1])
    for st in range(w4.steps):
        off, ids = wl.step_candidates(w4, st, device=dev, n_docs=n_docs)
        steps.append(gem.Cands(ids, off, max_list_len=w4.cands_per_step))
        rows = lens[ids.long()]
        pair_bytes += int(rows.sum().item()) * 132
        uniq = torch.unique(ids)
        uniq_bytes += int(lens[uniq.long()].sum().item()) * 132
    # the autotuner picks the gathered scorer's schedule for this step shape
    # (entries per wave, tiles in flight); every step has the same shape class
    gem.score_quant(Q8, D8, cands=steps[0])
    torch.cuda.synchronize()
    t_default = timed(lambda: gem.score_quant(Q8, D8, cands=steps[0]), 3)
    gsched, t_tuned = gem.autotune_gather(Q8, D8, steps[0], reps=3)
    log(f"expansion gather schedule {gsched}: {t_tuned:.3f} ms (library rule {t_default:.3f} ms)")
    eg = ExpansionGraph(Q8, D8, steps, ef=w4.ef)
    eg.capture()
    eg.replay()
    torch.cuda.synchronize()
    ms = timed(eg.replay, 3)
    per_step = ms / w4.steps
    r_ms = timed(lambda: eg.rerank(Q32, D32, 100), 1)
    pairs = sum(cc.ids.numel() for cc in steps)
    res = {"docs": n_docs, "doc_vectors": D32.n_vecs, "queries": Q32.n_sets, "steps": w4.steps, "ef": w4.ef,
           "cands_per_step": w4.cands_per_step, "ms_per_step": per_step,
           "pair_scores_per_s": pairs / (ms / 1e3),
           "gbps_per_pair_bytes": pair_bytes / w4.steps / (per_step / 1e3) / 1e9,
           "gbps_unique_bytes": uniq_bytes / w4.steps / (per_step / 1e3) / 1e9,
           "frac_of_hbm_peak_per_pair": pair_bytes / w4.steps / (per_step / 1e3) / PEAK_HBM,
           "rerank_f32_top100_ms": r_ms,
           "gather_schedule": dict(gsched, tuned_ms=t_tuned, library_rule_ms=t_default)}
    # the same gathered scorer on lists in which every document appears once
    # (a seeded permutation of the corpus cut into 4096 lists): per-pair bytes
    # are then unique bytes, so its rate is what a gather of distinct random
    # documents reaches, the ceiling for the step's 2.4 listings per document
    # when each listing has to read its document
    gp = torch.Generator(device="cpu").manual_seed(5001)
    perm = torch.randperm(n_docs, generator=gp).to(torch.int32).to(dev)
    per = n_docs // Q8.n_sets
    Cp = gem.Cands(perm[:per * Q8.n_sets].contiguous(), stride=per, n_lists=Q8.n_sets)
    bytes_p = int(lens[perm[:per * Q8.n_sets].long()].sum().item()) * 132
    gem.autotune_gather(Q8, D8, Cp, reps=3)
    t_p = timed(lambda: gem.score_quant(Q8, D8, cands=Cp), 5)
    res["distinct_docs_gather"] = {"lists": Q8.n_sets, "per_list": per, "bytes": bytes_p, "ms": t_p,
                                   "gbps": bytes_p / (t_p / 1e3) / 1e9,
                                   "frac_of_hbm_peak": bytes_p / (t_p / 1e3) / PEAK_HBM}
    log(f"gather of distinct documents: {bytes_p / 1e9:.2f} GB in {t_p:.3f} ms = {bytes_p / t_p / 1e6:.0f} GB/s")
    # MXFP4 rows: 64 bytes of codes + 4 exponent bytes per vector
    D4 = gem.quantize_mxfp4(D32)
    Q4 = gem.quantize_mxfp4(Q32)
    eg4 = ExpansionGraph(Q4, D4, steps, ef=w4.ef)
    eg4.capture()
    eg4.replay()
    torch.cuda.synchronize()
    ms4 = timed(eg4.replay, 3)
    b4 = eg4.beam.ids.cpu().numpy()
    a8 = eg.beam.ids.cpu().numpy()
    ov4 = np.mean([np.intersect1d(a8[i][a8[i] >= 0], b4[i][b4[i] >= 0]).size / w4.ef for i in range(a8.shape[0])])
    res["mxfp4"] = {"ms_per_step": ms4 / w4.steps, "speedup_vs_fp8_rows": per_step / (ms4 / w4.steps),
                    "gbps_per_pair_bytes": pair_bytes / 132 * 68 / w4.steps / (ms4 / w4.steps / 1e3) / 1e9,
                    "pair_scores_per_s": pairs / (ms4 / 1e3), "beam_overlap_with_fp8_rows": float(ov4)}
    log(f"mxfp4 expansion {ms4 / w4.steps:.3f} ms/step")
    del eg4, D4, Q4
    # MXFP6 rows: 96 bytes of codes + 4 exponent bytes per vector
    D6 = gem.quantize_mxfp6(D32)
    Q6 = gem.quantize_mxfp6(Q32)
    eg6 = ExpansionGraph(Q6, D6, steps, ef=w4.ef)
    eg6.capture()
    eg6.replay()
    torch.cuda.synchronize()
    ms6 = timed(eg6.replay, 3)
    b6 = eg6.beam.ids.cpu().numpy()
    ov6 = np.mean([np.intersect1d(a8[i][a8[i] >= 0], b6[i][b6[i] >= 0]).size / w4.ef for i in range(a8.shape[0])])
    res["mxfp6"] = {"ms_per_step": ms6 / w4.steps, "speedup_vs_fp8_rows": per_step / (ms6 / w4.steps),
                    "gbps_per_pair_bytes": pair_bytes / 132 * 100 / w4.steps / (ms6 / w4.steps / 1e3) / 1e9,
                    "pair_scores_per_s": pairs / (ms6 / 1e3), "beam_overlap_with_fp8_rows": float(ov6)}
    log(f"mxfp6 expansion {ms6 / w4.steps:.3f} ms/step")
    del eg6, D6, Q6

    # qCH expansion: the same steps with the corpus and the queries as codes
    # over an FP8 codebook (Secs. 4.2, 4.5): 4 bytes of code per vector
    # instead of its 132-byte FP8 row; the centroid rows are few enough to
    # stay in the caches
    log("expansion qCH: k-means codebook and corpus codes")
    C, Dc, qinfo = build_codebook(D32, n_iter=4, assign="bf16", seed=11, per_centroid=32)
    Dc8 = Dc.to_fp8()
    t_qenc, Qc = timed_once(lambda: gem.encode(Q32, C, assign="f32"))
    Qc8 = Qc.to_fp8()
    egq = ExpansionGraph(Qc8, Dc8, steps, ef=w4.ef)
    egq.capture()
    egq.replay()
    torch.cuda.synchronize()
    ms_q = timed(egq.replay, 3)
    a, b = eg.beam.ids.cpu().numpy(), egq.beam.ids.cpu().numpy()
    overlap = np.mean([np.intersect1d(a[i][a[i] >= 0], b[i][b[i] >= 0]).size / w4.ef for i in range(a.shape[0])])
    qinfo.update({"ms_per_step": ms_q / w4.steps, "speedup_vs_fp8_rows": per_step / (ms_q / w4.steps),
                  "query_encode_ms": t_qenc, "pair_scores_per_s": pairs / (ms_q / 1e3),
                  "code_bytes_per_step": pair_bytes / 132 * 4 / w4.steps,
                  "beam_overlap_with_fp8_rows": float(overlap)})
    res["qch"] = qinfo
    log(f"qCH expansion {ms_q / w4.steps:.3f} ms/step (FP8 rows {per_step:.3f})")
    del egq, Dc8, Dc, Qc8, Qc, C
    if not args.skip_cpu:
        # beam of a query subset against the oracle's replay of the same candidate lists
        import oracle
        ns = 8
        ok = 0
        bi = eg.beam.ids[:ns].cpu().numpy()
        bs = eg.beam.scores[:ns].double().cpu().numpy()
        qh = q.subset(list(range(ns)))
        qo = qh.offsets.cpu().numpy()
        codes, sc = oracle.quantize_fp8(qh.vecs.cpu().numpy())
        qd = oracle.dequantize_fp8(codes, sc)
        for i in range(ns):
            all_ids = torch.cat([cc.ids[cc.offsets[i]:cc.offsets[i + 1]] for cc in steps]).long()
            u = torch.unique(all_ids)
            starts, ln = c.offsets[u], lens[u]
            sub_off = torch.zeros(u.numel() + 1, dtype=torch.int64, device=dev)
            sub_off[1:] = torch.cumsum(ln, 0)
            rows = torch.repeat_interleave(starts - sub_off[:-1], ln) + torch.arange(int(sub_off[-1]), device=dev)
            sub_vecs = c.vecs[rows].cpu().numpy()
            dc, dsc = oracle.quantize_fp8(sub_vecs)
            est = oracle.ch_dense(qd[qo[i]:qo[i + 1]], [0, qo[i + 1] - qo[i]], oracle.dequantize_fp8(dc, dsc),
                                  sub_off.cpu().numpy())[0]
            u = u.cpu()
            full = np.full(n_docs, -np.inf)
            full[u.numpy()] = est
            tau = 2e-4 * max(abs(np.sort(est)[::-1][w4.ef - 1]), 1.0)
            good, _, _ = oracle.tie_aware_match(bi[i], full, w4.ef, tau)
            rel = np.abs(bs[i] - full[bi[i]]) / np.maximum(np.abs(full[bi[i]]), 1)
            ok += int(good and rel.max() <= 1e-4)
        res["beam_matches_oracle"] = f"{ok}/{ns} queries"
    return res



def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=2, choices=[2])
    ap.add_argument("--skip-cpu", action="store_true", help="skip the CPU oracle leg and recall")
    ap.add_argument("--cpu-sample", type=int, default=64,
                    help="query sets in the CPU-oracle sample (float64 check of the f32 path, oracle timing)")
    ap.add_argument("--shortlists", type=str, default="200,500,1000,2000",
                    help="shortlist lengths of the estimate -> rerank sweep")
    ap.add_argument("--skip-serving", action="store_true")
    ap.add_argument("--skip-expansion", action="store_true")
    ap.add_argument("--skip-graph", action="store_true", help="skip the graph-search leg (Alg. 5)")
    ap.add_argument("--only-graph", action="store_true", help="run the graph-search leg alone")
    ap.add_argument("--serve-rates", type=str, default="1000,2000,4000,8000,16000,32000",
                    help="comma-separated arrival rates (1/s)")
    ap.add_argument("--serve-requests", type=int, default=1500, help="minimum requests per rate")
    ap.add_argument("--serve-max-requests", type=int, default=20000, help="maximum requests per rate")
    ap.add_argument("--serve-shortlist", type=int, default=None,
                    help="FP8 shortlist reranked per serving request (default: the serving workload's)")
    ap.add_argument("--serve-shortlists", type=str, default="100,200,300,500,1000",
                    help="shortlist lengths whose recall is measured on the serving query mix")
    ap.add_argument("--serve-chunks", type=int, default=4,
                    help="corpus chunks of the serving loop (a request finishes after one pass over all of them)")
    ap.add_argument("--serve-chunk-work", type=int, default=8192,
                    help="query vectors x chunks an iteration may score (more chunks per iteration for light batches)")
    ap.add_argument("--serve-points-only", action="store_true",
                    help="serve the listed rates only (no memory-limited or 1000-shortlist comparison points)")
    ap.add_argument("--only-serving", action="store_true", help="run the serving leg alone (for profiling)")
    ap.add_argument("--dense-only", action="store_true",
                    help="run the bf16 / FP8 / MXFP4 dense scorers alone (for counter runs)")
    ap.add_argument("--tune-cache", type=str, default=None,
                    help="JSON tune cache: loaded before tuning and written with the schedules tuned here")
    ap.add_argument("--expand-docs", type=int, default=1_000_000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB copy kernel (reference for the HBM byte counters)")
    ap.add_argument("--only-expansion", action="store_true",
                    help="run the beam-expansion leg alone (for profiling); prints its result line")
    ap.add_argument("--only-rerank", action="store_true",
                    help="run the top-1000 rerank in every gather order alone (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.only_graph:
        print(json.dumps({"graph_search": bench_graph_search()}), flush=True)
        return
    if args.only_rerank:
        print(json.dumps({"rerank_orders": bench_rerank_orders(args)}), flush=True)
        return
    if args.only_expansion:
        res = bench_expansion(args)
        if args.copy_calibration:
            copy_calibration()
        print(json.dumps({"beam_expansion": res}), flush=True)
        return
    if args.tune_cache and os.path.exists(args.tune_cache):
        gem.load_tune_cache(args.tune_cache)
    if args.dense_only:
        res = bench_dense_only(args)
        if args.copy_calibration:
            copy_calibration()
        print(json.dumps({"dense": res}), flush=True)
        return
    if args.only_serving:
        w2 = wl.WORKLOADS[2]
        c_dev = wl.corpus(w2, device=torch.device("cuda:0"))
        D32 = gem.Sets(c_dev.vecs, c_dev.offsets, "f32", c_dev.max_len())
        line, keep = {}, (gem.quantize_fp8(D32), D32)
    else:
        line, keep = bench_exhaustive(args)
    if args.copy_calibration:
        copy_calibration()
    if not args.skip_serving:
        D8, D32 = keep
        sls = [int(x) for x in args.serve_shortlists.split(",") if x]
        if sls:
            line["serving_shortlist_recall"] = serving_shortlist_recall(D8, D32, sls)
        line["serving"] = []
        for ri, rate in enumerate([float(r) for r in args.serve_rates.split(",") if r]):
            log(f"serving at {rate:.0f} requests/s")
            # about 1.25 s of arrivals per rate, within the request bounds
            n_req = min(args.serve_max_requests, max(args.serve_requests, int(rate * 1.25)))
            line["serving"].append(bench_serving(D8, D32, rate=rate, n_req=n_req, rate_idx=ri,
                                               shortlist=args.serve_shortlist, chunk_work=args.serve_chunk_work,
                                               n_chunks=args.serve_chunks))
        if args.serve_rates and not args.serve_points_only:
            # a device-memory budget for 256 requests' state at 32,000/s: the
            # memory check, not the slot count, is what refuses requests
            log("serving at 32000 requests/s with a device budget of 256 requests")
            r = bench_serving(D8, D32, rate=32000.0, n_req=min(args.serve_max_requests, 20000), rate_idx=99,
                              max_resident=256, shortlist=args.serve_shortlist, n_chunks=args.serve_chunks,
                              chunk_work=args.serve_chunk_work)
            line["serving_memory_limited"] = r
            # the same offered load with the 1000-document shortlist of the
            # fixed-length rerank workload, for comparison
            log("serving at 16000 requests/s with a shortlist of 1000")
            line["serving_shortlist_1000"] = bench_serving(D8, D32, rate=16000.0,
                                                           n_req=min(args.serve_max_requests, 20000),
                                                           rate_idx=98, shortlist=1000, n_chunks=args.serve_chunks,
                                                           chunk_work=args.serve_chunk_work)
        if line["serving"]:
            # headline latency: the 2000/s point if swept, else the first rate
            ref = next((r for r in line["serving"] if r["rate_per_s"] == 2000.0), line["serving"][0])
            line["p50_ms"] = ref.get("p50_ms")
            line["p99_ms"] = ref.get("p99_ms")
            line["serving_rate_for_p50_p99"] = ref["rate_per_s"]
    del keep
    torch.cuda.empty_cache()
    if args.only_serving:
        print(json.dumps(line), flush=True)
        return
    if not args.skip_expansion:
        line["beam_expansion"] = bench_expansion(args)
        torch.cuda.empty_cache()
    if not args.skip_graph:
        line["graph_search"] = bench_graph_search()
    if args.tune_cache:
        gem.save_tune_cache(args.tune_cache)
        line["tune_cache"] = args.tune_cache
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
