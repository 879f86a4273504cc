"""Benchmark: kNN-graph build vectors/s on one MI355X, chosen form vs plain.

Workload (one GPU): N = 1,000,000 uint8 rows, d = 128, drawn from a mixture of
1000 Gaussians (centres U[0,200]^d, std 12, rounded and clipped to 0..255);
k-means into 16 shards with every row also in its second-nearest shard;
exact kNN K = 64 per shard, detour prune + reverse edges to R = 32, edge-union
merge to degree 64.  A step is one pass of the whole hot path over all 16
shards (16 x sg_knn_graph + 16 x sg_prune + sg_merge) on inputs resident in
HBM; partition and search are timed but outside the step.

Forms: plain = FP32 MFMA distances; the exact reduced forms are FP16 MFMA
(exact on uint8 rows with d <= 128) and INT8 MFMA on the rows shifted by -128
(exact INT32 sums); both give the plain graph bit for bit (recall 1.0), and the
faster one is the chosen form.  `value` is the chosen form's unique vectors per
second (N / step time); the other forms are timed the same way beside it.

Prints ONE JSON line.  --gpus above 1 is refused (one GPU per box here).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "f16": 2500.0, "bf16": 2500.0, "fp8": 5000.0, "i8": 5000.0}   # dense MFMA T(FL)OP/s


def cpu_model():
    """Host CPU model name (for the CPU-baseline record)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_step(sg, torch, Xcat, offs, K, R, prec, graphs, knn_all, mem_d, N):
    """One step of the headline: every shard's kNN graph and prune in one batched
    pass (persistent distance kernel over all shards' query blocks, largest
    shards first), then the merge over replicated vectors."""
    def step():
        sg.sg_knn_graph_batched(Xcat, offs, K, R, "l2", prec, out=(graphs, knn_all))
        return sg.sg_merge(offs, mem_d, graphs, R, N, 2 * R)
    return step


def build_per_shard_step(sg, shards, K, R, prec, graphs, nbrs, orders, mem_d, offs, N):
    """The same build as one distance launch and one prune per shard."""
    def step():
        for s, Xs in enumerate(shards):
            nb = nbrs[s]
            sg.sg_knn_graph(Xs, K, "l2", prec, out=(nb, None), order_out=orders[s])
            sg.sg_prune(nb, R, out=graphs[offs[s]:offs[s + 1]], order=orders[s])
        return sg.sg_merge(offs, mem_d, graphs, R, N, 2 * R)
    return step


def timed(torch, sg, step, steps, warmup):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    sg.sg_profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, launches = sg.sg_profile_end()
    return (t1 - t0) / steps, kms, launches, out


def calib_copy(torch, dev):
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def traffic_of(name, variant):
    """HBM bytes per distance-kernel launch from the committed counter record of
    this workload taken with the launch shape `variant` pinned, or None when
    there is none for that shape and the current kernel sources."""
    import glob
    from paper_2605_10135_amd import profiling
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "dist_topk_%s*_traffic.txt" % name))):
        rec = profiling.read_traffic(path)
        if rec is not None and rec["variant"] == variant:
            return rec
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--shards", type=int, default=16)
    ap.add_argument("--chosen", default="auto", choices=["auto", "f16", "i8", "fp32"],
                    help="exact form to report (auto: the faster of f16 and i8)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-per-shard", action="store_true",
                    help="skip the comparison with one distance launch and one prune per shard")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--force-variant", type=int, default=None,
                    help="after tuning, pin every distance launch to this launch-shape index "
                         "(counter runs use it to measure the shape a timed run chose)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--queries", type=int, default=10_000)
    ap.add_argument("--workload", default="sift1m",
                    choices=["sift1m", "precision", "batched", "learned", "partition", "degrees"])
    ap.add_argument("--oracle-rows", type=int, default=256,
                    help="rows per shard checked bit for bit against the FP64 oracle (0: no check)")
    ap.add_argument("--no-search", action="store_true", help="skip the search study")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip launch-shape tuning (with --force-variant: counter runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy 256 MiB device to device (scale for rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: each box here has one MI355X and the build is "
              "measured per GPU (shards are independent; see DESIGN.md for how it shards)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "precision":
        return run_precision(args)
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "learned":
        return run_learned(args)
    if args.workload == "partition":
        return run_partition(args)
    if args.workload == "degrees":
        return run_degrees(args)

    import torch

    import paper_2605_10135_amd as sg
    import synthdata

    dev = torch.device("cuda:0")
    if args.calib_copy:
        calib_copy(torch, dev)
    N, d, S, omega, K, R = args.n, 128, args.shards, 2, 64, 32
    t = time.perf_counter()
    X = synthdata.sift_like_u8(n=N, d=d, seed=1001)
    Q = synthdata.sift_like_u8(n=args.queries, d=d, seed=1001, stream=1)
    log("data %.1fs" % (time.perf_counter() - t))
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    init = synthdata.init_rows(N, S, seed=1001)

    # partition (outside the step)
    torch.cuda.synchronize()
    t = time.perf_counter()
    cent, prim, off, mem = sg.sg_partition(Xd, S, omega, 20, init)
    torch.cuda.synchronize()
    t_part = time.perf_counter() - t
    offs = [int(v) for v in off.tolist()]
    sizes = np.diff(offs)
    log("partition %.3fs sizes %s" % (t_part, sizes.tolist()))
    shards = [Xd[mem[offs[s]:offs[s + 1]].long()].contiguous() for s in range(S)]
    Xcat = Xd[mem.long()].contiguous()      # shard rows back to back (offsets offs)
    total = offs[-1]
    graphs = torch.empty((total, R), dtype=torch.int32, device=dev)
    knn_all = torch.empty((total, K), dtype=torch.int32, device=dev)
    flops = float(sum(2.0 * d * float(n) * float(n) for n in sizes))

    exact = ["f16", "i8"] if args.chosen == "auto" else [args.chosen]
    forms = exact + ([] if args.no_plain or "fp32" in exact else ["fp32"])
    # launch-shape autotuning (outside the timed region): the choice is recorded
    # per power-of-two bucket of shard size, so tune the largest shard of each
    # bucket present (the batched pass takes the choice of its largest shard)
    buckets = {}
    for i_, n_ in enumerate(sizes):
        b_ = int(n_).bit_length() - 1
        if b_ not in buckets or n_ > sizes[buckets[b_]]:
            buckets[b_] = i_
    tuned = {f: {b_: (sg.sg_knn_autotune(shards[i_], K, "l2", f) if not args.no_autotune else (0, []))
                 for b_, i_ in sorted(buckets.items())}
             for f in forms}
    # the batched pass itself is tuned per form (the persistent launch over all
    # shards can favour another shape than one launch of the largest shard)
    btuned = {f: (sg.sg_knn_graph_batched_autotune(Xcat, offs, K, R, "l2", f) if not args.no_autotune else (0, []))
              for f in forms}
    log("autotune %s batched %s" % (tuned, btuned))
    res = {}
    graph_of = {}
    if args.force_variant is not None:
        sg.sg_knn_force_variant(args.force_variant)
    for form in forms:
        step = build_step(sg, torch, Xcat, offs, K, R, form, graphs, knn_all, mem, N)
        sec, kms, launches, (mg, deg) = timed(torch, sg, step, args.steps, args.warmup)
        kavg = kms / max(launches, 1)
        ach = flops * args.steps / (kms / 1e3) / 1e12
        res[form] = dict(sec=sec, kernel_ms_total=kms, launches=launches, kernel_ms_avg=kavg,
                         tflops=ach, vps=N / sec, shard_rows_ps=total / sec,
                         variant=btuned[form][0])
        graph_of[form] = (mg.clone(), deg.clone(), knn_all.clone(), graphs.clone())
        log("%s: %.3f s/step, dist kernel %d launches, %.3f ms avg, %.1f TFLOP/s" % (
            form, sec, launches, kavg, ach))

    # the chosen form: the faster of the exact reduced forms (same graph)
    chosen = min(exact, key=lambda f: res[f]["sec"])
    variant = args.force_variant if args.force_variant is not None else res[chosen]["variant"]
    # stage breakdown of one chosen step (outside the timed region)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    e0, e1, e2 = ev(), ev(), ev()
    e0.record()
    sg.sg_knn_graph_batched(Xcat, offs, K, R, "l2", chosen, out=(graphs, knn_all))
    e1.record()
    mg, deg = sg.sg_merge(offs, mem, graphs, R, N, 2 * R)
    e2.record()
    torch.cuda.synchronize()
    stages = {"knn_and_prune_ms": e0.elapsed_time(e1), "merge_ms": e1.elapsed_time(e2)}

    # the integer passes on their own: the prune of all 2M shard rows as the
    # batched pass runs it (batch-row ids), and the merge; algorithmic bytes:
    # prune reads the K ids of a row and gathers K lists of K ids, then moves
    # about R x 20 B per row in the reverse pass; merge reads the shard graphs
    # and writes the merged one
    row0 = torch.repeat_interleave(torch.tensor(offs[:-1], dtype=torch.int32, device=dev),
                                   torch.tensor(sizes.tolist(), device=dev))
    knn_batch = (knn_all + row0[:, None]).contiguous()
    sg.sg_prune(knn_batch, R)
    e3, e4 = ev(), ev()
    e3.record()
    sg.sg_prune(knn_batch, R)
    e4.record()
    torch.cuda.synchronize()
    prune_ms = e3.elapsed_time(e4)
    # compulsory HBM bytes per row: the prune reads its K ids once, writes P,
    # each edge's reverse slot and its 32-bit reverse key, rereads P and the
    # keys to write F (4K + 24R + 24 with the counts and offsets; the reread
    # of the slots that places the few keys past a row's bucket is not
    # counted); the K lists of K ids it gathers per row are re-reads of the
    # same graph (cache hits), counted apart.  The merge reads each shard row's
    # R ids and member id and writes the merged rows and degrees.
    prune_bytes = float(total) * (4 * K + 24 * R + 24)
    gather_bytes = float(total) * 4 * K * K
    merge_bytes = float(total) * (R * 4 + 4) + float(N) * (2 * R * 4 + 4)
    integer_passes = {
        "prune": {"rows": total, "ms": prune_ms, "compulsory_bytes": prune_bytes,
                  "achieved_GBps": prune_bytes / (prune_ms / 1e3) / 1e9,
                  "frac_of_hbm_peak": prune_bytes / (prune_ms / 1e3) / 8e12,
                  "gathered_list_bytes": gather_bytes},
        "merge": {"rows": total, "ms": stages["merge_ms"], "compulsory_bytes": merge_bytes,
                  "achieved_GBps": merge_bytes / (stages["merge_ms"] / 1e3) / 1e9,
                  "frac_of_hbm_peak": merge_bytes / (stages["merge_ms"] / 1e3) / 8e12},
    }
    log("integer passes %s" % integer_passes)
    del knn_batch, row0

    # the same build with one distance launch and one prune per shard (same lists)
    per_shard = None
    if not args.no_per_shard:
        nbrs = [torch.empty((int(n), K), dtype=torch.int32, device=dev) for n in sizes]
        orders = [torch.empty(int(n), dtype=torch.int32, device=dev) for n in sizes]
        g1 = torch.empty_like(graphs)
        ps = build_per_shard_step(sg, shards, K, R, chosen, g1, nbrs, orders, mem, offs, N)
        ps_sec, ps_kms, ps_launches, (pmg, pdeg) = timed(torch, sg, ps, 2, 1)
        per_shard = {"ms_per_step": ps_sec * 1e3, "dist_launches_per_step": ps_launches // 2,
                     "dist_kernel_ms_per_step": ps_kms / 2,
                     "graph_identical_to_batched": bool(torch.equal(torch.cat(nbrs), graph_of[chosen][2])
                                                        and torch.equal(pmg, graph_of[chosen][0])
                                                        and torch.equal(pdeg, graph_of[chosen][1]))}
        log("per-shard launches: %.1f ms/step, identical %s" % (ps_sec * 1e3,
                                                                per_shard["graph_identical_to_batched"]))
        del nbrs, orders, g1

    same = None
    if "fp32" in graph_of and chosen != "fp32":
        a, b = graph_of[chosen], graph_of["fp32"]
        same = bool(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2]))
    same_exact = all(torch.equal(graph_of[f][0], graph_of[chosen][0]) and torch.equal(graph_of[f][2], graph_of[chosen][2])
                     for f in exact)

    search = search_study(torch, sg, Xd, Qd, mg, deg) if not args.no_search else None

    # exact check of the chosen kNN lists against the FP64 oracle: seeded rows
    # of every shard; the pruned graph of the smallest shard against the
    # oracle's prune of the GPU's own kNN lists
    import oracle
    rng = np.random.default_rng(5)
    t = time.perf_counter()
    rows_checked, rows_equal, knn_hits = 0, 0, 0
    X_h = X
    mem_h = mem.cpu().numpy()
    knn_h = graph_of[chosen][2].cpu().numpy()
    for s_ in range(S if args.oracle_rows > 0 else 0):
        Xs = X_h[mem_h[offs[s_]:offs[s_ + 1]]]
        Xs64 = oracle.widen(Xs)
        rows = rng.choice(Xs.shape[0], size=min(args.oracle_rows, Xs.shape[0]), replace=False)
        onbr, _ = oracle.knn(Xs64, K, rows=rows)
        g = knn_h[offs[s_]:offs[s_ + 1]][rows]
        rows_checked += len(rows)
        rows_equal += int((g == onbr).all(1).sum())
        knn_hits += sum(len(set(x_) & set(y_)) for x_, y_ in zip(g, onbr))
    s_small = int(np.argmin(sizes))
    a_, b_ = offs[s_small], offs[s_small + 1]
    prune_equal = (bool(np.array_equal(graph_of[chosen][3][a_:b_].cpu().numpy(), oracle.prune(knn_h[a_:b_], R)))
                   if args.oracle_rows > 0 else None)
    oracle_check = {"knn_rows_checked": rows_checked, "knn_rows_identical_to_oracle": rows_equal,
                    "knn_recall_at_64": knn_hits / float(max(rows_checked, 1) * K),
                    "pruned_graph_identical_to_oracle": {"shard": s_small, "rows": int(b_ - a_),
                                                         "identical": prune_equal},
                    "seconds": time.perf_counter() - t}
    log("oracle check %s" % oracle_check)

    # CPU baseline: the FP64 oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu:
        s0 = 0
        X0_64 = oracle.widen(X_h[mem_h[offs[s0]:offs[s0 + 1]]])
        n0 = X0_64.shape[0]
        oracle.knn(X0_64, K, rows=np.arange(2))          # warm-up (library load, thread start)
        nprobe = 4 * oracle.num_threads()
        probe = rng.choice(n0, size=nprobe, replace=False)
        t = time.perf_counter()
        oracle.knn(X0_64, K, rows=probe)
        per_row = (time.perf_counter() - t) / nprobe
        m = int(max(8, min(n0, args.cpu_seconds / max(per_row, 1e-9))))
        sample = rng.choice(n0, size=m, replace=False)
        t = time.perf_counter()
        oracle.knn(X0_64, K, rows=sample)
        dt = time.perf_counter() - t
        per_pair = dt / (m * n0)
        t_full = per_pair * float(sum(float(n) * float(n) for n in sizes))
        cpu = {"value": N / t_full, "unit": "vectors/s", "cores": oracle.num_threads(),
               "cpu_model": cpu_model(), "kind": "oracle",
               "sample": "exact FP64 kNN (K=64) of %d rows of shard 0 (%d rows, d=128) in %.1f s, "
                         "scaled by sum(n_s^2) to the full 16-shard kNN stage (prune and merge "
                         "not included, which favours the CPU)" % (m, n0, dt)}

    ch = res[chosen]
    prec = chosen
    traf = traffic_of("sift1m_u8_%s" % prec, variant)
    # algorithmic bytes: each shard's rows read once as operands, the K-list
    # of ids written once
    eb = {"fp32": 4, "f16": 2, "i8": 1}[prec]
    alg_bytes = float(sum(float(n) * (eb * d + 4 * K) for n in sizes))
    dtype_of = {"f16": "u8->f16 MFMA, f32 acc", "i8": "u8-128->i8 MFMA, i32 acc",
                "fp32": "u8->f32 MFMA, f32 acc"}
    line = {
        "metric": "kNN-graph build vectors/sec on 1 GPU at recall@k>=0.95; chosen vs plain",
        "value": ch["vps"],
        "unit": "vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ch["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_of[prec],
        "data": "synthetic",
        "config": {"workload": "N=1,000,000 x 128 u8 (1000-Gaussian mixture, centres U[0,200], "
                               "std 12), 16 overlapping k-means shards (omega=2), exact kNN K=64, "
                               "prune to R=32, merge to degree 64",
                   "form": prec, "n": N, "d": d, "shards": S, "K": K, "R": R,
                   "shard_rows": total},
        "roofline": {"bound": "mfma", "achieved": ch["tflops"], "peak": PEAK[prec],
                     "unit": "TOP/s" if prec == "i8" else "TFLOP/s", "frac": ch["tflops"] / PEAK[prec],
                     "traffic": traf["bytes"] if traf else None,
                     "traffic_unit": "bytes past L2 per launch (TCC FETCH_SIZE + WRITE_SIZE, copy-calibrated; "
                                     "mostly served by the MALL)",
                     "kernel": "dist_topk_batched_kernel (all 16 shards in one launch)",
                     "variant": variant,
                     "traffic_kernel": traf["kernels"] if traf else None,
                     "kernel_ms_avg": ch["kernel_ms_avg"],
                     "flops_per_launch_avg": flops * args.steps / max(ch["launches"], 1),
                     "algorithmic_bytes_per_launch_avg": alg_bytes * args.steps / max(ch["launches"], 1)},
        "cpu_baseline": cpu,
        "recall": {"knn_at_64_sampled": oracle_check["knn_recall_at_64"],
                   "knn_rows_identical_to_oracle": oracle_check["knn_rows_identical_to_oracle"]
                   == oracle_check["knn_rows_checked"],
                   "search_recall_at_10_L64": search["recall_at_10"]["64"] if search else None},
        "oracle_check": oracle_check,
        "search": search,
        "shard_rows_per_s": ch["shard_rows_ps"],
        "stages_ms": stages,
        "integer_passes": integer_passes,
        "per_shard_launches": per_shard,
        "forms": {f: {"value": res[f]["vps"], "ms_per_step": res[f]["sec"] * 1e3,
                      "kernel_ms_avg": res[f]["kernel_ms_avg"], "achieved": res[f]["tflops"],
                      "frac": res[f]["tflops"] / PEAK[f], "variant": res[f]["variant"]} for f in res},
        "exact_forms_identical": same_exact,
        "autotune": {f: {"2^%d" % b_: {"chosen": c, "variant_ms": t} for b_, (c, t) in v.items()}
                     for f, v in tuned.items()},
        "autotune_batched": {f: {"chosen": c, "variant_ms": t} for f, (c, t) in btuned.items()},
        "partition_s": t_part,
    }
    if "fp32" in res and prec != "fp32":
        pl = res["fp32"]
        line["plain"] = {"value": pl["vps"], "ms_per_step": pl["sec"] * 1e3,
                         "roofline_frac": pl["tflops"] / PEAK["fp32"], "achieved_tflops": pl["tflops"],
                         "kernel_ms_avg": pl["kernel_ms_avg"]}
        line["chosen_vs_plain"] = ch["vps"] / pl["vps"]
        line["chosen_graph_identical_to_plain"] = same
    print(json.dumps(line), flush=True)


def search_study(torch, sg, Xd, Qd, mg, deg, Ls=(16, 32, 64, 128, 256)):
    """Greedy-search recall@10 of the merged graph on the held-out queries for
    several beam widths, and the graph's reachability: the vertices reachable
    from the medoid entry, the weakly connected components, and the share of
    queries whose true nearest neighbour is reachable."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import breadth_first_order, connected_components

    xf = Xd.float()
    xn = (xf * xf).sum(1)
    gt, nn1 = [], []
    for a in range(0, Qd.shape[0], 256):
        qf = Qd[a:a + 256].float()
        dd = (qf * qf).sum(1, keepdim=True) + xn[None, :] - 2.0 * (qf @ xf.T)
        v, i = torch.topk(dd, 10, dim=1, largest=False)
        gt.append(v[:, -1])
        nn1.append(i[:, 0])
    kth, nn1 = torch.cat(gt), torch.cat(nn1)
    qf = Qd.float()
    rec, secs = {}, {}
    for L in Ls:
        t = time.perf_counter()
        ids, _ = sg.sg_search(Xd, mg, Qd, 10, L)
        torch.cuda.synchronize()
        secs[str(L)] = time.perf_counter() - t
        got = ids.long()
        dq = ((qf[:, None, :] - xf[got.clamp(min=0)]) ** 2).sum(-1)
        hits = ((dq <= kth[:, None]) & (got >= 0)).float().sum(1)
        rec[str(L)] = float((hits / 10.0).mean())
    # the medoid entry as the library picks it: the row nearest to the mean
    mean = Xd.double().mean(0).float()
    medoid = int(torch.argmin(((xf - mean[None, :]) ** 2).sum(1)).item())
    G = mg.cpu().numpy()
    n, w = G.shape
    src = np.repeat(np.arange(n), w)
    dst = G.ravel()
    ok = dst >= 0
    A = sp.csr_matrix((np.ones(int(ok.sum()), np.int8), (src[ok], dst[ok])), shape=(n, n))
    reach = breadth_first_order(A, medoid, directed=True, return_predecessors=False)
    reachable = np.zeros(n, bool)
    reachable[reach] = True
    ncomp, labels = connected_components(A, directed=True, connection="weak")
    nn1_h = nn1.cpu().numpy()
    return {"recall_at_10": rec, "seconds_10k_queries": secs, "medoid": medoid,
            "reachable_from_medoid": int(reachable.sum()), "n": n,
            "weak_components": int(ncomp),
            "largest_component": int(np.bincount(labels).max()),
            "queries_with_reachable_nn": float(reachable[nn1_h].mean()),
            "mean_degree": float(deg.float().mean().item())}


def run_precision(args):
    """Precision form: N = 4M unit-norm rows, d = 96, 2000-component mixture (std 0.15), IP;
    k-means into 13 shards with omega = 2; one GPU's share = shards 0..7 (~600k rows each);
    BF16 / FP8 distance keys with an FP32 re-rank of the top 128 (FP8 also of the top 256) to
    K = 64, prune to R = 32, merge; against the plain FP32 build of the same share.  The share's
    shards are built in one batched pass (re-rank included); the 256-wide re-rank, wider than the
    batched pass takes, runs shard by shard."""
    import torch

    import oracle
    import paper_2605_10135_amd as sg
    import synthdata

    dev = torch.device("cuda:0")
    N = args.n if args.n != 1_000_000 else 4_000_000
    d, S, omega, K, R, C = 96, 13, 2, 64, 32, 128
    share = 8
    t = time.perf_counter()
    X = synthdata.deep_like_unit(n=N, d=d, seed=1002)
    log("data %.1fs" % (time.perf_counter() - t))
    Xd = torch.from_numpy(X).to(dev)
    cent, prim, off, mem = sg.sg_partition(Xd, S, omega, 20, synthdata.init_rows(N, S, seed=1002))
    offs = [int(v) for v in off.tolist()]
    sizes = np.diff(offs)[:share]
    log("share sizes %s" % sizes.tolist())
    shards = [Xd[mem[offs[s]:offs[s + 1]].long()].contiguous() for s in range(share)]
    total = int(sizes.sum())
    soffs = [0] + np.cumsum(sizes).tolist()
    graphs = torch.empty((total, R), dtype=torch.int32, device=dev)
    mem_share = mem[:offs[share]]
    flops = float(sum(2.0 * d * float(n) * float(n) for n in sizes))

    Xshare = torch.cat(shards)               # the share's shard rows back to back (offsets soffs)
    knn_share = torch.empty((total, K), dtype=torch.int32, device=dev)

    def make_step(prec, rerank):
        # all shards of the share in one batched pass (re-rank included)
        def step():
            sg.sg_knn_graph_batched(Xshare, soffs, K, R, "ip", prec, out=(graphs, knn_share), rerank=rerank)
            return sg.sg_merge(soffs, mem_share, graphs, R, N, omega * R)
        return step

    # reduced forms: (name, precision, re-rank width); FP8 also with a wider
    # candidate list, which costs selection work but wins back recall.  Each
    # form's batched pass is tuned before it is timed.
    reduced = (("bf16", "bf16", C), ("fp8", "fp8", C), ("fp8_c256", "fp8", 2 * C))
    tuned = {f: sg.sg_knn_graph_batched_autotune(Xshare, soffs, K, R, "ip", prec_, rerank=rr_)
             for f, prec_, rr_ in reduced}
    log("autotune %s" % tuned)

    res, lists = {}, {}
    for form, prec, rr in reduced + (("fp32", "fp32", 0),):
        steps = args.steps if form != "fp32" else max(1, min(args.steps, 2))
        sec, kms, launches, _ = timed(torch, sg, make_step(prec, rr), steps, args.warmup)
        ach = flops * steps / (kms / 1e3) / 1e12
        res[form] = dict(sec=sec, vps=N * (share / S) / sec, shard_rows_ps=total / sec, tflops=ach,
                         frac=ach / PEAK[prec], kernel_ms_avg=kms / max(launches, 1), prec=prec, rerank=rr)
        lists[form] = [knn_share[soffs[i]:soffs[i] + 2000].clone() for i in range(2)]
        log("%s: %.3f s/step, %.1f TFLOP/s" % (form, sec, ach))

    # recall@64 of the reduced forms against the plain FP32 build (same shards, sampled rows)
    def rec(a, b):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        return float(np.mean([len(set(x) & set(y)) / K for x, y in zip(a, b)]))
    names = [f for f, _, _ in reduced]
    recall = {f: float(np.mean([rec(lists[f][i], lists["fp32"][i]) for i in range(2)])) for f in names}
    # error of each form against the FP64 oracle on 400 rows of shard 0: recall,
    # relative error of the returned distances against the FP64 distance of the
    # same pair, and the rows where some returned id is farther than the
    # oracle's K-th by more than the FP32 bound of the pair (a swap beyond the
    # tolerance); the bound is gamma_{d+1} sum_t |x_t y_t| per distance
    X0 = shards[0].cpu().numpy()
    X0_64 = oracle.widen(X0)
    rows = np.arange(0, 2000, 5)
    onbr, odist = oracle.knn(X0_64, K, oracle.IP, rows=rows)
    u = 2.0 ** -24
    gam = (d + 1) * u / (1 - (d + 1) * u)
    absx = np.abs(X0_64)

    def bound(r_, ids):
        return gam * (absx[r_][:, None, :] * absx[ids]).sum(-1)

    err = {}
    rr_of = {f: rr for f, _, rr in reduced}
    rr_of["fp32"] = 0
    prec_of = {f: p_ for f, p_, _ in reduced}
    prec_of["fp32"] = "fp32"
    for f in names + ["fp32"]:
        # the same lists as the batched pass (row-subset path), with distances
        gn, gdd = sg.sg_knn_rows(shards[0], rows, K, "ip", prec_of[f], rerank=rr_of[f])
        g, gd = gn.cpu().numpy(), gdd.cpu().numpy()
        same_lists = bool(np.array_equal(g, lists[f][0].cpu().numpy()[rows]))
        d64 = oracle.pair_dist(X0_64, np.repeat(rows[:, None], K, 1), g, oracle.IP)
        eg = bound(rows, g)
        eK = bound(rows, onbr[:, -1:])[:, 0]
        swapped = 0
        for r_ in range(len(rows)):
            extra = ~np.isin(g[r_], onbr[r_])
            if np.any(d64[r_][extra] > odist[r_, -1] + eg[r_][extra] + eK[r_]):
                swapped += 1
        e = {"recall_vs_fp64": float(np.mean([len(set(x) & set(y)) / K for x, y in zip(g, onbr)])),
             "max_abs_dist_err_vs_fp64": float(np.max(np.abs(np.sort(d64, 1) - odist))),
             "rows_swapped_beyond_fp32_bound": swapped / float(len(rows)), "rows": len(rows),
             "lists_equal_to_batched_pass": same_lists}
        rel = np.abs(gd.astype(np.float64) - d64) / np.maximum(np.abs(d64), 1e-6)
        e["max_rel_dist_err"] = float(rel.max())
        e["mean_rel_dist_err"] = float(rel.mean())
        err[f] = e

    # CPU baseline: the FP64 oracle (IP, d=96) on a bounded sample of shard 0,
    # scaled by sum(n_s^2) to the share's kNN stage
    cpu = None
    if not args.no_cpu:
        n0 = X0_64.shape[0]
        oracle.knn(X0_64, K, oracle.IP, rows=np.arange(2))
        nprobe = 4 * oracle.num_threads()
        t = time.perf_counter()
        oracle.knn(X0_64, K, oracle.IP, rows=np.arange(nprobe))
        per_row = (time.perf_counter() - t) / nprobe
        m = int(max(8, min(n0, args.cpu_seconds / max(per_row, 1e-9))))
        t = time.perf_counter()
        oracle.knn(X0_64, K, oracle.IP, rows=np.arange(m))
        dt = time.perf_counter() - t
        t_full = dt / (m * n0) * float(sum(float(n) * float(n) for n in sizes))
        cpu = {"value": N * (share / S) / t_full, "unit": "vectors/s", "cores": oracle.num_threads(),
               "cpu_model": cpu_model(), "kind": "oracle",
               "sample": "exact FP64 kNN (K=64, IP) of %d rows of shard 0 (%d rows, d=96) in %.1f s, scaled by "
                         "sum(n_s^2) to the share's kNN stage (prune and merge not included)" % (m, n0, dt)}
    chosen = max(names, key=lambda f: res[f]["vps"] if recall[f] >= 0.99 else -1)
    ch = res[chosen]
    cprec = ch["prec"]
    line = {
        "metric": "kNN-graph build vectors/sec on 1 GPU at recall@k>=0.95; chosen vs plain",
        "value": ch["vps"], "unit": "vectors/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ch["sec"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": cprec + " MFMA keys, f32 acc, f32 re-rank", "data": "synthetic",
        "config": {"workload": "N=4,000,000 x 96 unit-norm (2000-Gaussian mixture, std 0.15), IP, "
                               "13 k-means shards (omega=2), share = shards 0-7, top-%d by %s key, "
                               "FP32 re-rank to K=64, prune R=32, merge" % (ch["rerank"], cprec),
                   "shard_rows": total, "share_unique_vectors_est": N * share / S},
        "roofline": {"bound": "mfma", "achieved": ch["tflops"], "peak": PEAK[cprec], "unit": "TFLOP/s",
                     "frac": ch["frac"], "traffic": None, "kernel": "dist_topk",
                     "kernel_ms_avg": ch["kernel_ms_avg"]},
        "cpu_baseline": cpu,
        "forms": res, "recall_at_64_vs_plain": recall, "vs_fp64_oracle": err,
        "autotune": tuned,
        "chosen_vs_plain": ch["vps"] / res["fp32"]["vps"],
    }
    print(json.dumps(line), flush=True)


def _headline_data(args, torch, sg, synthdata, dev, n_comp=1000):
    """The headline rows, queries and seeded initial centroids (n_comp mixture
    components; 1000 for the headline workload)."""
    N, d, S = args.n, 128, args.shards
    X = synthdata.sift_like_u8(n=N, d=d, seed=1001, n_comp=n_comp)
    Q = synthdata.sift_like_u8(n=args.queries, d=d, seed=1001, stream=1, n_comp=n_comp)
    return (X, torch.from_numpy(X).to(dev), torch.from_numpy(Q).to(dev),
            synthdata.init_rows(N, S, seed=1001))


def _exact_build(torch, sg, Xd, mem, offs, K, R, N, prec, steps, warmup):
    """Batched exact build (kNN + prune) of the shards then the merge; returns
    (seconds per step, kernel ms per launch, merged graph, degrees, kNN lists,
    pruned graphs)."""
    dev = Xd.device
    Xcat = Xd[mem.long()].contiguous()
    total = int(offs[-1])
    graphs = torch.empty((total, R), dtype=torch.int32, device=dev)
    knn_all = torch.empty((total, K), dtype=torch.int32, device=dev)
    step = build_step(sg, torch, Xcat, offs, K, R, prec, graphs, knn_all, mem, N)
    sec, kms, launches, (mg, deg) = timed(torch, sg, step, steps, warmup)
    return sec, kms / max(launches, 1), mg, deg, knn_all, graphs


def run_partition(args):
    """Selectivity study (Sec. V-B, Algorithm 1; the paper's Table IV) on the
    headline workload: the rows are assigned block by block (64k-row blocks in
    row order, as a disk-resident set is read) with the blockwise-adaptive
    rule for epsilon in {1.1, 1.2, 1.5} and the original replicate-to-nearest
    rule (epsilon = inf); for each: the replica proportion (replicas / N, 100%
    for the original rule with omega = 2), the partition time, the exact build
    (batched kNN + prune + merge) and the search recall of the merged graph.
    Two data sets: the headline's 1000-component mixture (each shard then
    averages ~60 components, so a row's nearest and second-nearest shard
    centroids are at similar distances) and the same recipe with 64
    components (a few components per shard)."""
    import torch

    import paper_2605_10135_amd as sg
    import synthdata

    dev = torch.device("cuda:0")
    study = {}
    for n_comp in (1000, 64):
        study["components_%d" % n_comp] = _selectivity(args, torch, sg, synthdata, dev, n_comp)
    out = study["components_1000"]
    ch = out["eps_1.2"]
    line = {
        "metric": "kNN-graph build vectors/sec on 1 GPU at recall@k>=0.95; chosen vs plain",
        "value": ch["vectors_per_s"], "unit": "vectors/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ch["build_ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8-128->i8 MFMA, i32 acc", "data": "synthetic",
        "config": {"workload": "selectivity study: N=1,000,000 x 128 u8 (1000- and 64-Gaussian mixtures), 16 "
                               "shards, omega=2, blockwise-adaptive assignment in 65536-row blocks, epsilon in "
                               "{1.1, 1.2, 1.5, inf}, exact kNN K=64, prune R=32, merge; value = epsilon 1.2, "
                               "1000 components"},
        "roofline": None, "cpu_baseline": None,
        "selectivity": study,
        "chosen_vs_plain": ch["vectors_per_s"] / out["original"]["vectors_per_s"],
    }
    print(json.dumps(line), flush=True)


def _selectivity(args, torch, sg, synthdata, dev, n_comp):
    X, Xd, Qd, init = _headline_data(args, torch, sg, synthdata, dev, n_comp)
    N, S, omega, K, R = args.n, args.shards, 2, 64, 32
    prec = "i8"
    out = {}
    for name, eps, tau0 in (("original", float("inf"), 1.0), ("eps_1.5", 1.5, 1.5), ("eps_1.2", 1.2, 1.5),
                            ("eps_1.1", 1.1, 1.5)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        cent, prim, off, mem = sg.sg_partition_blockwise(Xd, S, omega, 20, init, epsilon=eps, tau0=tau0,
                                                         block_rows=65536, shard_cap=0, adaptive=True)
        torch.cuda.synchronize()
        t_part = time.perf_counter() - t
        offs = [int(v) for v in off.tolist()]
        sizes = np.diff(offs)
        # tune the launch shape on the largest shard of each size bucket
        buckets = {}
        for i_, n_ in enumerate(sizes):
            b_ = int(n_).bit_length() - 1
            if b_ not in buckets or n_ > sizes[buckets[b_]]:
                buckets[b_] = i_
        sg.sg_knn_graph_batched_autotune(Xd[mem.long()].contiguous(), offs, K, R, "l2", prec)
        sec, kms, mg, deg, _, _ = _exact_build(torch, sg, Xd, mem, offs, K, R, N, prec, args.steps, args.warmup)
        search = search_study(torch, sg, Xd, Qd, mg, deg, Ls=(64, 128))
        out[name] = {"epsilon": eps, "tau0": tau0, "shard_rows": int(offs[-1]),
                     "replica_proportion": (offs[-1] - N) / float(N * (omega - 1)),
                     "partition_s": t_part, "build_ms_per_step": sec * 1e3, "dist_kernel_ms": kms,
                     "vectors_per_s": N / sec, "search_recall_at_10": search["recall_at_10"],
                     "reachable_from_medoid": search["reachable_from_medoid"],
                     "weak_components": search["weak_components"], "shard_sizes": sizes.tolist()}
        log("%d components, %s: %s" % (n_comp, name, {k: v for k, v in out[name].items() if k != "shard_sizes"}))
    return out


def run_degrees(args):
    """The paper's default and stress degree settings (degree R from K
    candidates: 64 from 128, 128 from 256) on the headline workload: exact
    batched build, prune and merge; seeded rows of every shard and the pruned
    graph of the smallest shard checked against the oracle."""
    import torch

    import oracle
    import paper_2605_10135_amd as sg
    import synthdata

    dev = torch.device("cuda:0")
    X, Xd, Qd, init = _headline_data(args, torch, sg, synthdata, dev)
    N, S, omega, d = args.n, args.shards, 2, 128
    cent, prim, off, mem = sg.sg_partition(Xd, S, omega, 20, init)
    offs = [int(v) for v in off.tolist()]
    sizes = np.diff(offs)
    mem_h = mem.cpu().numpy()
    flops = float(sum(2.0 * d * float(n) * float(n) for n in sizes))
    out = {}
    for K, R in ((64, 32), (128, 64), (256, 128)):
        res = {}
        for prec in ("f16", "i8"):
            sg.sg_knn_graph_batched_autotune(Xd[mem.long()].contiguous(), offs, K, R, "l2", prec)
            sec, kms, mg, deg, knn_all, graphs = _exact_build(torch, sg, Xd, mem, offs, K, R, N, prec,
                                                              args.steps, args.warmup)
            res[prec] = (sec, kms)
            log("K=%d R=%d %s: %.1f ms/step, dist %.1f ms" % (K, R, prec, sec * 1e3, kms))
        prec = min(res, key=lambda p_: res[p_][0])
        sec, kms, mg, deg, knn_all, graphs = _exact_build(torch, sg, Xd, mem, offs, K, R, N, prec, 1, 0)
        rng = np.random.default_rng(K)
        knn_h = knn_all.cpu().numpy()
        checked = equal = 0
        for s_ in range(S):
            Xs64 = oracle.widen(X[mem_h[offs[s_]:offs[s_ + 1]]])
            rows = rng.choice(Xs64.shape[0], size=min(64, Xs64.shape[0]), replace=False)
            onbr, _ = oracle.knn(Xs64, K, rows=rows)
            checked += len(rows)
            equal += int((knn_h[offs[s_]:offs[s_ + 1]][rows] == onbr).all(1).sum())
        s_small = int(np.argmin(sizes))
        a_, b_ = offs[s_small], offs[s_small + 1]
        prune_ok = bool(np.array_equal(graphs[a_:b_].cpu().numpy(), oracle.prune(knn_h[a_:b_], R)))
        search = search_study(torch, sg, Xd, Qd, mg, deg, Ls=(64, 128))
        out["%d/%d" % (R, K)] = {
            "K": K, "R": R, "form": prec, "ms_per_step": res[prec][0] * 1e3, "vectors_per_s": N / res[prec][0],
            "dist_kernel_ms": res[prec][1], "dist_achieved": flops / (res[prec][1] / 1e3) / 1e12,
            "forms_ms_per_step": {p_: v[0] * 1e3 for p_, v in res.items()},
            "knn_rows_checked": checked, "knn_rows_identical_to_oracle": equal,
            "pruned_graph_identical_to_oracle": {"shard": s_small, "rows": int(b_ - a_), "identical": prune_ok},
            "search_recall_at_10": search["recall_at_10"]}
        log("%d/%d: %s" % (R, K, out["%d/%d" % (R, K)]))
    ch = out["64/128"]
    line = {
        "metric": "kNN-graph build vectors/sec on 1 GPU at recall@k>=0.95; chosen vs plain",
        "value": ch["vectors_per_s"], "unit": "vectors/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ch["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "exact u8 MFMA (%s)" % ch["form"], "data": "synthetic",
        "config": {"workload": "degree settings R/K = 32/64, 64/128, 128/256 on N=1,000,000 x 128 u8, "
                               "16 shards (omega=2), exact batched build + prune + merge; value = 64/128"},
        "roofline": None, "cpu_baseline": None, "degrees": out,
    }
    print(json.dumps(line), flush=True)


def laion_like_gpu(torch, N, d, n_comp, sigma, seed, dev):
    """N unit-norm FP16 rows from an n_comp-component Gaussian mixture (centres
    N(0, I), std sigma), drawn on the GPU with a seeded generator and ordered
    by (component, draw index)."""
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    mu = torch.randn((n_comp, d), generator=g, device=dev)
    comp = torch.randint(0, n_comp, (N,), generator=g, device=dev)
    order = torch.sort(comp, stable=True).indices
    comp = comp[order]
    X = torch.empty((N, d), dtype=torch.float16, device=dev)
    for a in range(0, N, 1 << 20):
        b = min(N, a + (1 << 20))
        x = mu[comp[a:b]] + sigma * torch.randn((b - a, d), generator=g, device=dev)
        X[a:b] = (x / x.norm(dim=1, keepdim=True)).half()
    return X


def run_batched(args):
    """Batching form: 64 shards with lognormal sizes (ln 1e5, 0.8) clipped to
    [20k, 500k], overlapping windows (each shard shares ~25% with the next) over
    ~6M unit-norm FP16 rows of dimension 768 from a 4000-component mixture,
    inner product, K = 64, R = 32; all shards built by one captured batched
    pass (sg_knn_graph_batched replaying its plan), then merged; against 64
    sequential single-shard builds of the same shards."""
    import torch

    import oracle
    import paper_2605_10135_amd as sg
    import synthdata

    dev = torch.device("cuda:0")
    d, K, R = 768, 64, 32
    sizes = synthdata.batched_shard_sizes(64, seed=1003)
    N, offs, mem = synthdata.overlapping_windows(sizes)
    t = time.perf_counter()
    U = laion_like_gpu(torch, N, d, 4000, 0.15, 1003, dev)
    memd = torch.from_numpy(mem).to(dev)
    X = U[memd.long()].contiguous()                  # shard rows, concatenated
    torch.cuda.synchronize()
    log("data %.1fs: N=%d, shard rows %d" % (time.perf_counter() - t, N, int(offs[-1])))
    total = int(offs[-1])
    flops = float(sum(2.0 * d * float(n) * float(n) for n in sizes))
    graphs = torch.empty((total, R), dtype=torch.int32, device=dev)
    knn = torch.empty((total, K), dtype=torch.int32, device=dev)
    stream = torch.cuda.Stream()
    plan = sg.BatchPlan()
    tuned = sg.sg_knn_graph_batched_autotune(X, offs, K, R, "ip", "f16")
    log("autotune (batched pass) %s" % (tuned,))

    def batched_step():
        with torch.cuda.stream(stream):
            sg.sg_knn_graph_batched(X, offs, K, R, "ip", "f16", out=(graphs, knn), stream=stream, plan=plan)
            out = sg.sg_merge(offs, memd, graphs, R, N, 2 * R, stream=stream)
        return out

    knn_p = torch.empty_like(knn)
    graphs_p = torch.empty_like(graphs)

    def plain_step():
        with torch.cuda.stream(stream):
            for s_ in range(len(sizes)):
                a, b = int(offs[s_]), int(offs[s_ + 1])
                sg.sg_knn_graph(X[a:b], K, "ip", "f16", out=(knn_p[a:b], None), stream=stream)
                sg.sg_prune(knn_p[a:b], R, out=graphs_p[a:b], stream=stream)
            out = sg.sg_merge(offs, memd, graphs_p, R, N, 2 * R, stream=stream)
        return out

    def timed_on(step, steps, warmup):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, out

    sec_b, (mg, deg) = timed_on(batched_step, args.steps, args.warmup)
    log("batched: %.3f s/step" % sec_b)
    # distance-kernel time of the batched pass: one eager (uncaptured) run
    torch.cuda.synchronize()
    sg.sg_profile_begin()
    with torch.cuda.stream(stream):
        sg.sg_knn_graph_batched(X, offs, K, R, "ip", "f16", out=(graphs, knn), stream=stream)
    torch.cuda.synchronize()
    kms, launches = sg.sg_profile_end()
    steps_p = max(1, min(args.steps, 2))
    sec_p, (mg_p, deg_p) = timed_on(plain_step, steps_p, 1)
    log("per-shard: %.3f s/step" % sec_p)
    same = bool(torch.equal(knn, knn_p) and torch.equal(graphs, graphs_p) and torch.equal(mg, mg_p))

    # sampled rows of the smallest shard against the FP64 oracle
    s0 = int(np.argmin(sizes))
    a, b = int(offs[s0]), int(offs[s0 + 1])
    Xs = X[a:b].cpu().numpy()
    rows = np.random.default_rng(3).choice(b - a, size=32, replace=False)
    X64 = oracle.widen(Xs)
    onbr, _ = oracle.knn(X64, K, oracle.IP, rows=rows)
    g = knn[a:b].cpu().numpy()[rows]
    rec = float(np.mean([len(set(x) & set(y)) / K for x, y in zip(g, onbr)]))

    cpu = None
    if not args.no_cpu:
        oracle.knn(X64, K, oracle.IP, rows=np.arange(2))  # warm-up (library load, thread start)
        nprobe = 4 * oracle.num_threads()
        t = time.perf_counter()
        oracle.knn(X64, K, oracle.IP, rows=np.arange(nprobe))
        per_row = (time.perf_counter() - t) / nprobe / (b - a)
        m = int(max(8, min(b - a, args.cpu_seconds / max(per_row * (b - a), 1e-9))))
        t = time.perf_counter()
        oracle.knn(X64, K, oracle.IP, rows=np.arange(m))
        dt = time.perf_counter() - t
        per_pair = dt / (m * (b - a))
        t_full = per_pair * float(sum(float(n) * float(n) for n in sizes))
        cpu = {"value": total / t_full, "unit": "shard rows/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "exact FP64 kNN (K=64, IP) of %d rows of the smallest shard (%d rows, d=768) in %.1f s, "
                         "scaled by sum(n_s^2) to the 64-shard kNN stage (prune and merge not included)"
                         % (m, b - a, dt)}
    ach = flops / (kms / 1e3) / 1e12 if kms > 0 else None
    line = {
        "metric": "kNN-graph build vectors/sec on 1 GPU at recall@k>=0.95; chosen vs plain",
        "value": total / sec_b, "unit": "shard rows/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec_b * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16 MFMA, f32 acc", "data": "synthetic",
        "config": {"workload": "64 shards, sizes lognormal(ln 1e5, 0.8) clipped [20k, 500k] (seed 1003), "
                               "overlapping windows (25%%) over N=%d unit-norm FP16 rows, d=768, 4000-component "
                               "mixture, IP, K=64, R=32, one captured batched pass + merge" % N,
                   "shard_rows": total, "N_unique": N, "flops": flops},
        "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK["f16"], "unit": "TFLOP/s",
                     "frac": ach / PEAK["f16"] if ach else None, "traffic": None, "kernel": "dist_topk_batched",
                     "kernel_ms": kms, "launches": launches},
        "cpu_baseline": cpu,
        "unique_vectors_per_s": N / sec_b,
        "plain": {"value": total / sec_p, "ms_per_step": sec_p * 1e3,
                  "what": "64 sequential sg_knn_graph + sg_prune calls, then sg_merge"},
        "chosen_vs_plain": sec_p / sec_b,
        "batched_identical_to_per_shard": same,
        "recall_at_64_vs_fp64_oracle_32_rows": rec,
    }
    plan.close()
    print(json.dumps(line), flush=True)


def l1_nonneg_gpu(torch, N, d, n_comp, sigma, seed, dev):
    """N rows |mu_c + sigma * N(0, I)| (centres N(0, I), n_comp components),
    each scaled to unit L1 norm; drawn on the GPU with a seeded generator."""
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    mu = torch.randn((n_comp, d), generator=g, device=dev)
    comp = torch.randint(0, n_comp, (N,), generator=g, device=dev)
    X = torch.empty((N, d), dtype=torch.float32, device=dev)
    for a in range(0, N, 1 << 19):
        b = min(N, a + (1 << 19))
        x = (mu[comp[a:b]] + sigma * torch.randn((b - a, d), generator=g, device=dev)).abs()
        X[a:b] = x / x.sum(dim=1, keepdim=True)
    return X


def run_learned(args):
    """Learned form: N = 2M FP32 rows, d = 960, |500-component mixture, std 0.2|
    L1-normalised, L2.  Exact K = 64 lists of 200k anchors (FP32 plain kernel)
    train an MLP 960 -> 256 -> 64 (GELU, BF16 products, FP32 masters) for 2000
    Adam steps of 1024 in-batch pairs; every row is projected, FP8 scores on the
    unit projections propose 256 candidates, an exact FP32 re-rank keeps 64,
    prune to R = 32.  A 10k-row sample judged by exact lists gates the result
    (recall@64 >= 0.95, else the plain build is used).  Gain test on the same
    sample: trained vs untrained net vs a random projection at c = 256."""
    import torch

    import oracle
    import paper_2605_10135_amd as sg

    dev = torch.device("cuda:0")
    N = args.n if args.n != 1_000_000 else 2_000_000
    d, H, E, K, R, c = 960, 256, 64, 64, 32, 256
    n_anchor, n_gate, steps_t, B = min(200_000, N // 4), min(10_000, N // 8), 2000, 1024
    t = time.perf_counter()
    X = l1_nonneg_gpu(torch, N, d, 500, 0.2, 1004, dev)
    torch.cuda.synchronize()
    log("data %.1fs" % (time.perf_counter() - t))
    rng = np.random.default_rng(1004)
    perm = rng.permutation(N)
    anchors, sample = perm[:n_anchor], perm[n_anchor:n_anchor + n_gate]

    def sync_time(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    # 1. training labels: exact lists of the anchors
    t_lab, (lab, _) = sync_time(lambda: sg.sg_knn_rows(X, anchors, K, "l2", "fp32"))
    log("labels %.2fs" % t_lab)
    # 2. training
    gt = torch.Generator().manual_seed(1004)
    W1 = torch.randn((H, d), generator=gt) * (2.0 / d) ** 0.5
    W2 = torch.randn((E, H), generator=gt) * (1.0 / H) ** 0.5
    b1 = torch.randn(H, generator=gt) * 0.01
    b2 = torch.randn(E, generator=gt) * 0.01
    mu, sigma = sg.sg_mlp_stats(X, anchors)
    mk = lambda: sg.MLP(*(t_.to(dev) for t_ in (W1, b1, W2, b2)), mu, sigma)
    net, net0 = mk(), mk()
    a_idx = rng.integers(0, n_anchor, size=B * steps_t)
    pos = lab.cpu().numpy()[a_idx, rng.integers(0, K, size=B * steps_t)]
    t_train, losses = sync_time(lambda: sg.sg_mlp_train(X, net, anchors[a_idx], pos, B, steps_t, lr=1e-3))
    lo = losses.cpu().numpy()
    log("train %.2fs loss %.3f -> %.3f" % (t_train, lo[:20].mean(), lo[-20:].mean()))

    # 3. the learned build (timed)
    def learned_step():
        F = sg.sg_mlp_project(X, net)
        nbr, _ = sg.sg_knn_graph_learned(X, F, c, K, dist=False)
        return nbr, sg.sg_prune(nbr, R)
    for _ in range(args.warmup):
        learned_step()
    t_build, (nbr, graph) = sync_time(learned_step)
    log("learned build %.2fs" % t_build)

    # 4. gate on the sample
    t_gate, (ex, _) = sync_time(lambda: sg.sg_knn_rows(X, sample, K, "l2", "fp32"))
    exh = ex.cpu().numpy()
    rec = lambda lists: float(np.mean([len(set(a) & set(b)) / K for a, b in zip(lists, exh)]))
    r_learned = rec(nbr.cpu().numpy()[sample])
    accepted = r_learned >= 0.95

    # 5. gain test: candidate recall at the same budget c (equals recall after the exact re-rank)
    def proposals(P):
        cand, _ = sg.sg_knn_rows(P.contiguous(), sample, c, "ip", "fp8")
        return rec_c(cand.cpu().numpy())
    rec_c = lambda cand: float(np.mean([len(set(a) & set(b)) / K for a, b in zip(cand, exh)]))
    G = torch.randn((d, E), generator=torch.Generator().manual_seed(7)).to(dev)
    gain = {"trained": proposals(sg.sg_mlp_project(X, net)),
            "untrained": proposals(sg.sg_mlp_project(X, net0)),
            "random_projection": proposals(torch.nn.functional.normalize(X @ G, dim=1))}
    log("gate recall %.4f gain %s" % (r_learned, gain))

    # 6. the plain build: exact FP32 kNN + prune (fallback and comparator)
    t_plain = None
    plain_rec = None
    plain_kms = None
    if not args.no_plain or not accepted:
        sg.sg_profile_begin()
        t_plain, (pn, pg) = sync_time(lambda: (lambda nb: (nb, sg.sg_prune(nb, R)))(
            sg.sg_knn_graph(X, K, "l2", "fp32", dist=False)[0]))
        plain_kms, _ = sg.sg_profile_end()
        plain_rec = rec(pn.cpu().numpy()[sample])
        log("plain build %.2fs (distance kernel %.1f ms)" % (t_plain, plain_kms))
    # CPU baseline: the FP64 oracle (L2, d=960) on a bounded sample of rows
    # against all N, scaled to N rows
    cpu = None
    if not args.no_cpu:
        X64 = oracle.widen(X.cpu().numpy())
        oracle.knn(X64, K, rows=np.arange(2))
        t = time.perf_counter()
        oracle.knn(X64, K, rows=sample[:4 * oracle.num_threads()])
        per_row = (time.perf_counter() - t) / (4 * oracle.num_threads())
        m = int(max(8, min(len(sample), args.cpu_seconds / max(per_row, 1e-9))))
        t = time.perf_counter()
        oracle.knn(X64, K, rows=sample[:m])
        dt = time.perf_counter() - t
        cpu = {"value": m / dt, "unit": "vectors/s", "cores": oracle.num_threads(), "cpu_model": cpu_model(),
               "kind": "oracle",
               "sample": "exact FP64 kNN (K=64, L2) of %d of the %d rows (d=960) in %.1f s; rows/s of the kNN "
                         "stage (prune not included)" % (m, N, dt)}
        del X64
    t_end = t_lab + t_train + t_build + t_gate
    if not accepted:
        t_end += t_plain
    line = {
        "metric": "kNN-graph build vectors/sec on 1 GPU at recall@k>=0.95; chosen vs plain",
        "value": N / t_end, "unit": "vectors/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
        "ms_per_step": t_end * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 MLP, fp8 scoring, f32 re-rank", "data": "synthetic",
        "config": {"workload": "N=%d x 960 FP32 (|500-component mixture, std 0.2|, L1-normalised), L2; "
                               "MLP 960-256-64 trained 2000 x 1024 on exact lists of %d anchors; FP8 proposals "
                               "c=256, FP32 re-rank K=64, prune R=32; %d-row recall gate" % (N, n_anchor, n_gate)},
        "roofline": ({"bound": "mfma", "achieved": 2.0 * d * float(N) * float(N) / (plain_kms / 1e3) / 1e12,
                      "peak": PEAK["fp32"], "unit": "TFLOP/s",
                      "frac": 2.0 * d * float(N) * float(N) / (plain_kms / 1e3) / 1e12 / PEAK["fp32"],
                      "traffic": None, "kernel": "dist_topk_kstream (the plain FP32 build, which the gate chose)"
                      if not accepted else "dist_topk_kstream (the plain FP32 comparator)",
                      "kernel_ms": plain_kms} if plain_kms else None),
        "cpu_baseline": cpu,
        "accepted": accepted,
        "recall_at_64_gate_sample": r_learned,
        "gain_candidate_recall_c256": gain,
        "seconds": {"labels": t_lab, "train": t_train, "learned_build": t_build, "gate": t_gate,
                    "plain_build": t_plain},
        "learned_build_only_vectors_per_s": N / t_build,
        "plain": {"value": N / t_plain if t_plain else None, "recall_gate_sample": plain_rec},
        "chosen_vs_plain": (t_plain / t_end) if t_plain else None,
        "train_loss_first_last": [float(lo[:20].mean()), float(lo[-20:].mean())],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
