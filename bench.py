"""Benchmark of the Panther hot path on one MI355X.

One step = one pass of the whole hot path over the workload: sample R
weighted random paths of length T (walk kernel), build the vertex-to-path
index, and answer every query's top-k in the batched form.  Inputs are
resident in device memory before the timed region starts.  The headline
value is path-steps/s (R * T per step).  Also reported: batched vs plain
top-k queries/s (with a bit-exactness check between the two), per-stage
device times, the walk kernel's roofline figure and the oracle timed on the
host cores on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat20]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def walk_algorithmic_bytes(R, T):
    """Bytes the guide-table walk must move per launch: per step a 16-byte
    vertex record, a 4-byte guide entry, one 8-byte {prefix, column} record
    and the 4-byte vertex written; per path the 4-byte start-set read and
    the 4-byte start vertex written."""
    return R * (T * (16 + 4 + 8 + 4) + 8)


def cpu_baseline(g, queries, T, k, seed, R_sample):
    import oracle

    oracle.build()
    t0 = time.perf_counter()
    paths = oracle.walk(g, T, R_sample, seed)
    inv_ptr, inv_pid = oracle.index(g.n, paths)
    oracle.topk(g.n, paths, inv_ptr, inv_pid, queries, k)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": R_sample * T / dt, "unit": "path-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": (f"oracle walk of {R_sample} paths (T={T}) + index + top-{k} of all "
                       f"{len(queries)} queries on that index, {dt:.2f} s")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat20")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="paths in the oracle sample (0 = the full R of the workload)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: multi-GPU sharding is designed, not built "
              "(see DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1504_02577_amd import inputs
    from paper_1504_02577_amd.panther import Panther

    os.environ.setdefault("PANTHER_INPUT_CACHE", "/tmp/panther_inputs")
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
    P.set_option("topk.form", 0)
    tp = time.perf_counter()
    P.topk(dq, k, out=out, stream=stream)
    torch.cuda.synchronize()
    tp = time.perf_counter() - tp
    plain = tuple(t.cpu().numpy() for t in out)
    exact = all((a == b).all() for a, b in zip(batched, plain))
    P.set_option("topk.form", 1)

    walk_ms = float(np.mean(stage["walk"]))
    walk_bytes = walk_algorithmic_bytes(R, T)
    achieved = walk_bytes / (walk_ms * 1e-3) / 1e9

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
                               f"{nq} queries, k={k}",
                   "parallelism": "single GPU"},
        "stage_ms": {kk: float(np.mean(v)) for kk, v in stage.items()},
        "topk_batched_qps": nq / tb,
        "topk_plain_qps": nq / tp,
        "batched_vs_plain": tp / tb,
        "batched_equals_plain": bool(exact),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_walk", "algorithmic_bytes_per_launch": walk_bytes,
                     "kernel_ms": walk_ms},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        res["cpu_baseline"] = cpu_baseline(g, q, T, k, seed, args.cpu_sample or R)
    P.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
