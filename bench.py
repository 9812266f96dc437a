"""Throughput of the matrix-element hot path on one MI355X.

Workload: g g -> t tbar g g at sqrt(s) = 13 TeV, 2^20 seeded RAMBO points
(seed 2), float64 momenta resident in HBM.  One step = one evaluation of
|M|^2 for every point (all helicities, diagrams and colour sums).

Prints one JSON line: MEs/s, the roofline of the dominant kernel (measured
with HIP events on the launch stream) and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nevt", type=int, default=1 << 20)
    ap.add_argument("--process", default="gg_ttgg")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=1 << 13, help="events for the CPU oracle baseline")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2503_21935_amd as me
    from inputs import process_points

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    mom_np = process_points(args.process, args.nevt, args.seed)
    print(f"[bench] generated {args.nevt} points in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    mom = torch.from_numpy(mom_np).to(dev)
    out = torch.empty(args.nevt, dtype=torch.float64, device=dev)
    m = me.MatrixElement(args.process)
    info = m.info()
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        m.eval(mom, out=out, stream=stream)
    torch.cuda.synchronize()

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        m.eval(mom, out=out, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    kernel_ms = ev0.elapsed_time(ev1) / args.steps  # one launch per step
    ms_per_step = wall * 1e3 / args.steps
    value = args.nevt / (ms_per_step * 1e-3)

    flops_evt = info["flops_per_event"]
    achieved = flops_evt * args.nevt / (kernel_ms * 1e-3) / 1e12
    res = out.cpu().numpy()
    assert np.all(np.isfinite(res)), "non-finite results"

    line = {
        "metric": "matrix elements/sec, gg->ttgg 1 GPU (FP64 exact kernel)",
        "value": value,
        "unit": "MEs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded RAMBO points, sqrt(s)=13 TeV",
        "config": {"workload": f"{args.process} |M|^2, {args.nevt} RAMBO points seed {args.seed}, "
                               f"{info['nhel_good']} helicities, {info['ndiag']} diagrams, "
                               f"{info['ncol']}x{info['ncol']} colour matrix",
                   "nevt": args.nevt, "parallelism": "single GPU, one event per lane"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "flops_per_event": flops_evt, "kernel_ms": kernel_ms},
    }

    if not args.no_cpu:
        import oracle

        n = min(args.cpu_sample, args.nevt)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        c0 = time.perf_counter()
        ref = oracle.me2(args.process, mom_np[:n])
        cpu_s = time.perf_counter() - c0
        rel = np.abs(res[:n] / ref - 1)
        line["cpu_baseline"] = {"value": n / cpu_s, "unit": "MEs/s", "cores": threads, "kind": "oracle",
                                "sample": f"first {n} of the {args.nevt} points, float64 oracle "
                                          f"(colour-ordered Berends-Giele), {cpu_s:.1f} s"}
        line["max_rel_dev_vs_oracle_on_sample"] = float(rel.max())
    m.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
