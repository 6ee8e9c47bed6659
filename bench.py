"""Benchmark of the Panther hot path on one MI355X.

One step = one pass of the whole hot path over the workload: sample R
weighted random paths of length T (walk kernel), build the vertex-to-path
index, and answer every query's top-k in the batched form.  Inputs are
resident in device memory before the timed region starts.  The headline
value is path-steps/s (R * T per step) on R-MAT scale 24 (T=5, R=10^8, 10^5
degree-weighted queries, k=50), the largest configuration that is one GPU's
whole job.  Also reported: batched vs plain top-k queries/s (with a
bit-exactness check between the two), per-stage device times and their
fractions of the HBM roofline by algorithmic bytes, the dominant kernel's
roofline object, and the oracle timed on the host cores on a bounded sample
of the same workload.

Other workloads (one JSON line each, not the headline):
  --workload rmat20     the same step at R-MAT scale 20 (R = 10^7, 10^4 queries)
  --workload rmat22_pp  Panther++: features (D=50) and 65,536 kNN queries
                        (k=20) in the BF16 matrix-core form, FP64 form timed
                        on a 1,024-query subset
  --workload serve      continuous-batching server under Poisson arrivals on
                        the R-MAT 24 state (--serve-graph rmat20 for the
                        smaller one)
  --workload allv       all-vertex top-5 (every vertex of the graph is a
                        query, the paper's Table 2 workload) on --allv-graph
  --workload bigR       R-MAT 24 with R from the sample-size bound for
                        eps = sqrt(1/|E|) (Theorem 1, about 8.6e8 paths, more
                        than 2^32 index entries): one sampling + index step,
                        the 10^5-query batch, and a sampled check of paths and
                        lists against the oracle
  --workload twocopy    cross-graph Panther++ between R-MAT 20 and a copy
                        with permuted ids (each with its own paths): 65,536
                        degree-weighted queries, k=10, D=50, and how often a
                        vertex's twin is in its top-10

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat24]
"""
import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def walk_algorithmic_bytes(P, g, T):
    """Bytes the walk must move per launch (Algorithm 3 with the inverse-CDF
    step of Eq. 3), from the sampled paths: per step leaving vertex v, its
    row bounds (8 B), ceil(log2 d_v) probes of 4-byte weight prefixes, the
    chosen column (4 B) and the vertex written (4 B); per path, the start-set
    entry read (4 B) and the start written (4 B)."""
    import torch

    deg = torch.from_numpy(np.diff(g.row_ptr.astype(np.int64))).cuda()
    # ceil(log2 d) for d >= 1 (0 for d = 1): bit length of d - 1
    probes = torch.zeros_like(deg)
    x = (deg - 1).clamp(min=0)
    while bool((x > 0).any()):
        probes += (x > 0).to(torch.int64)
        x >>= 1
    paths = P.paths_device()
    R = paths.shape[0]
    total_probes = 0
    for t in range(T):
        total_probes += int(probes[paths[:, t].to(torch.int64)].sum().item())
    del paths
    return R * T * 16 + 4 * total_probes + R * 8, total_probes / (R * T)


def index_algorithmic_bytes(R, T, nnz, n):
    """Read every path row (4 B per vertex), write every list entry (4 B)
    and the list offsets (8 B per vertex)."""
    return 4 * R * (T + 1) + 4 * nnz + 8 * (n + 1)


def count_algorithmic_bytes(lens, k):
    """Per query: its two list offsets (16 B), per listed path its id (4 B)
    and its 24-byte row (6 vertices), and k (id, count) pairs written."""
    return int(16 * len(lens) + 28 * int(np.sum(lens)) + 8 * k * len(lens))


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    import hashlib

    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[kernel][workload]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
            return None
        return rec["hbm_bytes_per_launch"]
    except (OSError, KeyError, ValueError, TypeError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(g, queries, T, k, seed, R_sample):
    """The oracle on a bounded sample of the workload: R_sample paths walked
    and indexed on one thread, then all queries answered on that index with
    every host thread.  Value in path-steps/s of the sample."""
    import oracle

    oracle.build()
    all_threads = oracle.get_threads()
    oracle.set_threads(1)
    t0 = time.perf_counter()
    paths = oracle.walk(g, T, R_sample, seed)
    t_walk = time.perf_counter() - t0
    t0 = time.perf_counter()
    inv_ptr, inv_pid = oracle.index(g.n, paths)
    t_index = time.perf_counter() - t0
    oracle.set_threads(all_threads)
    t0 = time.perf_counter()
    oracle.topk(g.n, paths, inv_ptr, inv_pid, queries, k)
    t_q = time.perf_counter() - t0
    dt = t_walk + t_index + t_q
    return {"value": R_sample * T / dt, "unit": "path-steps/s", "cores": all_threads,
            "kind": "oracle",
            "sample": (f"oracle on {R_sample} of the workload's paths (same graph, seed, T): "
                       f"walk {t_walk:.2f} s and index {t_index:.2f} s on 1 thread, then top-{k} "
                       f"of all {len(queries)} queries on that index {t_q:.2f} s on "
                       f"{all_threads} threads; total {dt:.2f} s"),
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"walk_path_steps_per_s": R_sample * T / t_walk,
                              "index_entries_per_s": len(inv_pid) / t_index},
            "all_threads": {"queries_per_s": len(queries) / t_q, "threads": all_threads}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat24")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain-form comparison (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=50_000.0)
    ap.add_argument("--serve-graph", default="rmat24")
    ap.add_argument("--allv-graph", default="rmat20")
    ap.add_argument("--allv-k", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="paths in the oracle sample (0 = R/50)")
    args = ap.parse_args()
    if args.workload == "serve":
        # one hardware queue per stream (the context's, the batched form's
        # second stream, three lanes, torch's): 4 per process would put two
        # lanes on one queue and serialise them
        os.environ["GPU_MAX_HW_QUEUES"] = "8"
    if args.gpus != 1:
        print("bench.py runs on one GPU only: multi-GPU sharding is designed, not built; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1504_02577_amd import inputs
    from paper_1504_02577_amd.panther import Panther

    os.environ.setdefault("PANTHER_INPUT_CACHE", "/tmp/panther_inputs")
    if args.calibrate_copy:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del x, y
    if args.workload == "rmat22_pp":
        return bench_pp(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "allv":
        return bench_allv(args)
    if args.workload == "twocopy":
        return bench_twocopy(args)
    if args.workload == "bigR":
        return bench_bigR(args)
    t0 = time.time()
    g, q, p = inputs.workload(args.workload)
    T, R, seed, k = p["T"], p["R"], p["seed"], p["k"]
    log(f"workload {args.workload}: n={g.n} m={g.m} T={T} R={R} queries={len(q)} k={k} "
        f"(inputs {time.time() - t0:.1f} s)")

    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(0)
    log(f"device: {props.name} CUs={props.multi_processor_count} "
        f"mem={props.total_memory / 2**30:.0f} GiB "
        f"lds/block={getattr(props, 'shared_memory_per_block', '?')}")
    P = Panther(0)
    P.load_graph(g)
    P.set_option("timing", 1)
    dq = torch.from_numpy(q).to(dev)
    nq = len(q)
    out = (torch.empty((nq, k), dtype=torch.int32, device=dev),
           torch.empty((nq, k), dtype=torch.uint32, device=dev),
           torch.empty(nq, dtype=torch.int32, device=dev))
    stream = torch.cuda.current_stream().cuda_stream

    def step():
        P.sample_paths(T, R, seed)
        P.topk(dq, k, out=out, stream=stream)

    P.set_option("topk.form", 1)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tune_file = os.environ.get("PANTHER_TUNE_CACHE") or os.path.join(
        os.environ.get("HOME", "/tmp"), ".cache", "panther_tune.txt")
    if os.path.exists(tune_file):
        with open(tune_file) as f:
            tuned = [ln.split() for ln in f if ln.startswith(f"gfx950:n{g.n}:T{T}:R{R}:")]
        if tuned:
            log("batched configuration (block, wgs/CU, tier B divisor, bucket bias): "
                + " ".join(tuned[-1][1:]))
    stage = {"walk": [], "index": [], "topk": []}
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
        st = P.stage_times()  # waits for this step's events
        for key in stage:
            stage[key].append(st[key])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = R * T * args.steps / elapsed
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step")

    # batched vs plain top-k (same paths), bit-exactness between the two
    batched = tuple(t.cpu().numpy().copy() for t in out)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    P.topk(dq, k, out=out, stream=stream)
    torch.cuda.synchronize()
    tb = time.perf_counter() - tb
    tp, exact = None, None
    if not args.no_plain:
        P.set_option("topk.form", 0)
        tp = time.perf_counter()
        P.topk(dq, k, out=out, stream=stream)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        plain = tuple(t.cpu().numpy() for t in out)
        exact = all((a == b).all() for a, b in zip(batched, plain))
        P.set_option("topk.form", 1)

    # algorithmic bytes of each stage and their fractions of the HBM peak
    walk_ms = float(np.mean(stage["walk"]))
    index_ms = float(np.mean(stage["index"]))
    topk_ms = float(np.mean(stage["topk"]))
    walk_bytes, mean_probes = walk_algorithmic_bytes(P, g, T)
    nnz = P.nnz()
    ptr, _ = P.index_device(g.n)
    lens = (ptr[1:] - ptr[:-1]).cpu().numpy()[q]
    del ptr, _
    idx_bytes = index_algorithmic_bytes(R, T, nnz, g.n)
    cnt_bytes = count_algorithmic_bytes(lens, k)

    def frac(b, ms):
        gbs = b / (ms * 1e-3) / 1e9
        return {"ms": ms, "algorithmic_bytes": int(b), "GBps": gbs, "frac": gbs / HBM_PEAK_GBS}

    stages = {"walk": frac(walk_bytes, walk_ms), "index": frac(idx_bytes, index_ms),
              "count_topk": frac(cnt_bytes, topk_ms)}
    stages["walk"]["mean_probes_per_step"] = mean_probes
    stages["count_topk"]["sum_list_rows"] = int(np.sum(lens))
    achieved = stages["walk"]["GBps"]

    res = {
        "metric": "path-steps/s",
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: R-MAT scale {int(math.log2(g.n))}, "
                               f"{g.m} CSR entries, lognormal weights, T={T}, R={R}, "
                               f"{nq} queries ({p['queries'][0]}), k={k}",
                   "parallelism": "single GPU"},
        "stage_ms": {kk: float(np.mean(v)) for kk, v in stage.items()},
        "stages": stages,
        "topk_batched_qps": nq / tb,
        "topk_plain_qps": nq / tp if tp else None,
        "batched_vs_plain": tp / tb if tp else None,
        "batched_equals_plain": exact,
        # the longest single launch of a step is the walk (k_walk32, one
        # launch); the top-k stage is several shorter hub launches
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("k_walk32", args.workload),
                     "kernel": "k_walk32", "algorithmic_bytes_per_launch": int(walk_bytes),
                     "kernel_ms": walk_ms},
    }
    # achievable HBM bandwidth on this machine: a 2 GiB device-to-device copy
    # (2 GiB read + 2 GiB written), best of 4, timed with HIP events
    copy_gbs = measured_copy_gbs()
    res["roofline"]["measured_copy_GBps"] = copy_gbs
    res["roofline"]["frac_of_measured_copy"] = achieved / copy_gbs if copy_gbs else None
    P.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        res["cpu_baseline"] = cpu_baseline(g, q, T, k, seed, args.cpu_sample or R // 50)
    print(json.dumps(res), flush=True)


def measured_copy_gbs():
    import torch

    x = torch.empty(1 << 29, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    best = None
    for _ in range(4):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del x, y
    return 2.0 * (1 << 31) / (best * 1e-3) / 1e9


def bench_allv(args):
    """All-vertex top-k: one call answers the top-k of every vertex."""
    import torch
    from paper_1504_02577_amd import inputs
    from paper_1504_02577_amd.panther import Panther

    g, _, p = inputs.workload(args.allv_graph)
    T, R, seed, k = p["T"], p["R"], p["seed"], args.allv_k
    P = Panther(0)
    P.load_graph(g)
    P.set_option("timing", 1)
    P.sample_paths(T, R, seed)
    dev = torch.device("cuda:0")
    out = (torch.empty((g.n, k), dtype=torch.int32, device=dev),
           torch.empty((g.n, k), dtype=torch.uint32, device=dev),
           torch.empty(g.n, dtype=torch.int32, device=dev))
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(args.warmup):
        P.topk_all(g.n, k, out=out, stream=stream)
    torch.cuda.synchronize()
    dev_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P.topk_all(g.n, k, out=out, stream=stream)
        dev_ms.append(P.stage_times()["topk"])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    res = {"metric": "vertices/s", "value": g.n / dt, "unit": "vertices/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic",
           "config": {"workload": f"allv: top-{k} of all {g.n} vertices of {args.allv_graph}, "
                                  f"T={T}, R={R}", "parallelism": "single GPU"},
           "device_ms": float(np.mean(dev_ms)), "roofline": None}
    if not args.no_cpu_baseline:
        import oracle

        oracle.build()
        paths = oracle.walk(g, T, R, seed)
        inv_ptr, inv_pid = oracle.index(g.n, paths)
        sample = min(g.n, 200_000)
        t1 = time.perf_counter()
        oracle.topk(g.n, paths, inv_ptr, inv_pid, np.arange(sample, dtype=np.int32), k)
        dt1 = time.perf_counter() - t1
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        res["cpu_baseline"] = {"value": sample / dt1, "unit": "vertices/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"oracle top-{k} of vertices 0..{sample - 1} on the "
                                         f"oracle's own paths and index, {dt1:.2f} s"}
    P.close()
    print(json.dumps(res), flush=True)


def bench_bigR(args):
    """Sample-size-driven R at R-MAT 24: R = sample_size(sqrt(1/|E|), 0.5,
    0.1, T) paths, nnz above 2^32."""
    import torch
    import oracle
    from paper_1504_02577_amd import inputs
    from paper_1504_02577_amd.panther import Panther, panther_sample_size

    g, q, p = inputs.workload("rmat24")
    T, seed, k = p["T"], p["seed"], p["k"]
    E = g.m // 2
    R = int(panther_sample_size(math.sqrt(1.0 / E), 0.5, 0.1, T))
    log(f"bigR: |E| = {E}, R = {R}")
    P = Panther(0)
    P.load_graph(g)
    P.set_option("timing", 1)
    steps = max(1, args.steps)
    stage = {"walk": [], "index": []}
    t0 = time.perf_counter()
    for _ in range(steps):
        P.sample_paths(T, R, seed)
        st = P.stage_times()
        for kk in stage:
            stage[kk].append(st[kk])
    dt = (time.perf_counter() - t0) / steps
    nnz = P.nnz()
    dq = torch.from_numpy(q).cuda()
    out = (torch.empty((len(q), k), dtype=torch.int32, device="cuda"),
           torch.empty((len(q), k), dtype=torch.uint32, device="cuda"),
           torch.empty(len(q), dtype=torch.int32, device="cuda"))
    stream = torch.cuda.current_stream().cuda_stream
    P.topk(dq, k, out=out, stream=stream)
    torch.cuda.synchronize()
    tq = time.perf_counter()
    P.topk(dq, k, out=out, stream=stream)
    torch.cuda.synchronize()
    tq = time.perf_counter() - tq
    # sampled parity: paths of random ids against the oracle's own walk of
    # those ids; lists of sampled vertices against a scan of all paths
    oracle.build()
    rng = np.random.default_rng(17)
    pids = np.sort(rng.integers(0, R, 4096))
    want = oracle.walk_pids(g, T, seed, pids)
    paths = P.paths_device()
    got = paths[torch.from_numpy(pids).cuda()].cpu().numpy()
    paths_ok = bool((got == want).all())
    ptr, pid = P.index_device(g.n)
    vs = np.concatenate([q[:4], rng.integers(0, g.n, 4)]).astype(np.int64)
    lists_ok = True
    for v in vs.tolist():
        a, b = int(ptr[v]), int(ptr[v + 1])
        lst = pid[a:b].to(torch.int64)
        has = (paths == v).any(1)
        lists_ok &= int(has.sum()) == b - a
        if b > a:
            lists_ok &= bool((lst[1:] > lst[:-1]).all()) and bool(has[lst].all())
    del paths, ptr, pid
    res = {"metric": "path-steps/s", "value": R * T / dt, "unit": "path-steps/s", "n_gpus": 1,
           "steps": steps, "warmup": 0, "ms_per_step": dt * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": f"bigR: R-MAT 24, R = {R} from the sample-size bound with "
                                  f"eps = sqrt(1/|E|), |E| = {E}, T={T}; step = sampling + index",
                      "parallelism": "single GPU"},
           "stage_ms": {kk: float(np.mean(v)) for kk, v in stage.items()}, "nnz": int(nnz),
           "topk_batched_ms": tq * 1e3, "topk_queries": len(q),
           "sampled_paths_equal_oracle": paths_ok, "sampled_lists_valid": bool(lists_ok),
           "roofline": None}
    P.close()
    print(json.dumps(res), flush=True)


def bench_twocopy(args):
    """Cross-graph Panther++ on two copies of one graph (identity resolution)."""
    import torch
    from paper_1504_02577_amd import inputs
    from paper_1504_02577_amd.panther import Panther

    g, _, p = inputs.workload("rmat20")
    gb, perm = inputs.permuted_copy(g, 4)
    T, R, D, k = p["T"], p["R"], 50, 10
    A = Panther(0)
    B = Panther(0)
    A.load_graph(g)
    B.load_graph(gb)
    A.sample_paths(T, R, 1)
    B.sample_paths(T, R, 2)
    # degree-weighted queries: vertices whose path lists are long enough for
    # their features to tell them apart (most low-degree vertices share
    # identical few-count features at this R)
    q = inputs.queries_by_degree(g, 65_536, 107)
    t0 = time.perf_counter()
    A.features(g.n, D)
    B.features(gb.n, D)
    feat_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        A.pp_topk_cross(B, q, D, k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ids, dist = A.pp_topk_cross(B, q, D, k)
    dt = (time.perf_counter() - t0) / args.steps
    twin = perm[q]
    rate10 = float(np.mean((ids == twin[:, None]).any(1)))
    rate1 = float(np.mean(ids[:, 0] == twin))
    res = {"metric": "cross-graph Panther++ queries/s", "value": len(q) / dt,
           "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16+f64", "data": "synthetic",
           "config": {"workload": f"twocopy: R-MAT 20 and a copy with permuted ids, T={T}, "
                                  f"R={R} each, {len(q)} degree-weighted queries, k={k}, "
                                  f"D={D}"},
           "twin_in_top1": rate1, "twin_in_top10": rate10, "features_s_both": feat_s,
           "roofline": None}
    A.close()
    B.close()
    print(json.dumps(res), flush=True)


def bench_pp(args):
    """Panther++ at R-MAT 22: feature pass and BF16-MFMA kNN (+ FP64 rerank)."""
    import torch
    from paper_1504_02577_amd import inputs
    from paper_1504_02577_amd.panther import Panther

    t0 = time.time()
    g, q, p = inputs.workload("rmat22_pp")
    T, R, seed, k, D = p["T"], p["R"], p["seed"], p["k"], p["D"]
    log(f"workload rmat22_pp: n={g.n} m={g.m} R={R} queries={len(q)} D={D} k={k} "
        f"(inputs {time.time() - t0:.1f} s)")
    P = Panther(0)
    P.load_graph(g)
    P.set_option("timing", 1)
    P.sample_paths(T, R, seed)
    P.set_option("pp.form", 1)
    P.set_option("pp.pool", p["pool"])
    dq = torch.from_numpy(q).cuda()
    out = (torch.empty((len(q), k), dtype=torch.int32, device="cuda"),
           torch.empty((len(q), k), dtype=torch.float64, device="cuda"))
    stream = torch.cuda.current_stream().cuda_stream
    P.pp_topk(dq, D, k, out=out, stream=stream)  # builds theta, warms up
    torch.cuda.synchronize()
    feat_ms = P.stage_times()["features"]  # first pass: includes growing the scratch
    # steady state: resampling drops theta, the next call rebuilds it with
    # the scratch already in place
    P.sample_paths(T, R, seed)
    P.pp_topk(dq, D, k, out=out, stream=stream)
    torch.cuda.synchronize()
    feat_steady_ms = P.stage_times()["features"]
    times = []
    for _ in range(max(1, args.steps)):
        t = time.perf_counter()
        P.pp_topk(dq, D, k, out=out, stream=stream)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    pp_ms = P.stage_times()["pp"]
    err, rec = P.pp_stats()
    cert_nq, cert_redo = P.pp_certified()
    bf16_ids = out[0].cpu().numpy()
    sub = q[:1024]
    P.set_option("pp.form", 0)
    t = time.perf_counter()
    fids, fdist = P.pp_topk(sub, D, k)
    fp64_s = time.perf_counter() - t
    agree = float((fids == bf16_ids[:1024]).mean())
    # products actually computed by the pool pass (the norm-band search
    # skips the rest), each a 64-term bf16 dot product
    scanned = P.pp_scanned()
    flops = 2.0 * len(q) * g.n * scanned * 64
    achieved = flops / (pp_ms * 1e-3) / 1e12
    res = {
        "metric": "Panther++ queries/s", "value": len(q) / min(times), "unit": "queries/s",
        "n_gpus": 1, "steps": len(times), "warmup": 1, "ms_per_step": 1e3 * min(times),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f64",
        "data": "synthetic",
        "config": {"workload": f"rmat22_pp: R-MAT scale 22, {g.m} CSR entries, T={T}, R={R}, "
                               f"D={D}, {len(q)} queries, k={k}, pool {p['pool']}"},
        "features_ms": feat_ms, "features_steady_ms": feat_steady_ms, "pp_kernels_ms": pp_ms,
        "pre_rerank_recall": rec, "bf16_max_rel_err": err,
        "certified_queries": cert_nq - cert_redo, "recomputed_exactly": cert_redo,
        "pool_scanned_fraction": scanned,
        "fp64_form_queries_per_s": len(sub) / fp64_s,
        "fp64_vs_bf16_id_agreement_1024": agree,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": achieved / 2500.0, "traffic": None,
                     "kernel": "k_pp_pool + k_pp_rerank",
                     "algorithmic_flops_per_launch": flops, "kernel_ms": pp_ms},
    }
    P.close()
    print(json.dumps(res), flush=True)


def bench_serve(args):
    """Continuous batching under Poisson arrivals: 80% Panther / 20%
    Panther++, k uniform over {10, 50, 200}, query vertices proportional to
    degree."""
    from paper_1504_02577_amd import inputs
    from paper_1504_02577_amd.panther import Panther, Server

    g, _, p = inputs.workload(args.serve_graph)
    T, R, seed = p["T"], p["R"], p["seed"]
    P = Panther(0)
    P.load_graph(g)
    P.sample_paths(T, R, seed)
    log(f"serve: {args.serve_graph} n={g.n} R={R}; building features ...")
    srv = Server(P, mem_budget_bytes=1 << 32, max_batch=2048, lanes=3, D=50)
    rng = np.random.default_rng(5)
    n_req = int(args.serve_rate * args.serve_seconds)
    qs = inputs.queries_by_degree(g, n_req, 6)
    kinds = (rng.random(n_req) < 0.2).astype(np.int32)
    ks = rng.choice([10, 50, 200], n_req).astype(np.int32)
    gaps = rng.exponential(1.0 / args.serve_rate, n_req)
    arrive = np.cumsum(gaps)
    got = 0
    t0 = time.perf_counter()
    i = 0
    while i < n_req:
        now = time.perf_counter() - t0
        while i < n_req and arrive[i] <= now:
            srv.submit(int(kinds[i]), int(qs[i]), int(ks[i]), i)
            i += 1
        got += len(srv.poll(0))
    while got < n_req and time.perf_counter() - t0 < arrive[-1] + 60:
        got += len(srv.poll(10000))
    st = srv.stats()
    mem = srv.memory()
    srv.stop()
    P.close()
    res = {"metric": "p99 ms", "value": st["p99_ms"], "unit": "ms", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": None, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32+bf16+f64",
           "data": "synthetic",
           "config": {"workload": f"serve: {args.serve_graph}, R={R}, Poisson "
                                  f"{args.serve_rate:.0f}/s for {args.serve_seconds:.0f} s, "
                                  "80% Panther / 20% Panther++ (D=50), k in {10,50,200}, "
                                  "3 lanes, max batch 2048"},
           "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "sustained_qps": st["qps"],
           "offered_qps": args.serve_rate, "completed": st["completed"], "submitted": n_req,
           "lane_share_bytes": mem["lane_share_bytes"], "peak_lane_bytes": mem["peak_lane_bytes"]}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
