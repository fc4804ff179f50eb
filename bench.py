"""Throughput benchmark of the dense optical-flow estimator on one MI355X.

One step = the whole estimator (normalisation, pyramid, every Gauss-Newton
iteration at every level, up-sampling) on one synthetic image pair already
resident in device memory.  Default workload: 1024x1024 12-bit pair
(translation 1.37, -0.62 px plus a 0.01 px/px shear), 4 levels, window
radius 5, 4 iterations per level, normalisation radius 1, float32 storage.

Prints one JSON line.  ``roofline`` covers the dominant kernel (the fused
Gauss-Newton iteration at full resolution): algorithmic bytes per launch
(per-sweep model: both images + flow in + flow out per pixel) over its
average launch duration, timed with HIP events on the stream it runs on.
``cpu_baseline`` times the FP64 CPU oracle on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="shear_1mp", choices=["shear_1mp", "rankine_256", "paper_1mp"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of replaying a hipGraph")
    ap.add_argument("--variant", default="tuned", choices=["tuned", "auto", "march", "tile64x32", "tile64x16"],
                    help="Gauss-Newton work decomposition: autotuned per level (default) or forced")
    ap.add_argument("--kernel-launches", type=int, default=200, help="launches timed for the dominant kernel")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def workload(name):
    import synth
    if name == "shear_1mp":
        pair, prm = synth.config_shear_1mp()
        desc = "1024x1024 12-bit particle pair, translation (1.37,-0.62) px + 0.01 px/px shear"
        bits = 12
    elif name == "rankine_256":
        pair, prm = synth.config_rankine_256()
        desc = "256x256 8-bit particle pair, Rankine vortex R=32 D=3"
        bits = 8
    else:
        pair, prm = synth.config_paper_sweep(1024, 1024, 3, 0)
        desc = "1024x1024 8-bit particle pair, paper throughput setting NR=2 KR=10 IT=3 PSL=2"
        bits = 8
    return pair, prm, desc, bits


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this estimator build has no multi-GPU path "
              "(independent pairs shard across GPUs with no communication); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2509_25924_amd as ofv
    from paper_2509_25924_amd import _build

    if not _build.built():
        _build.build()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    ofv.load()
    dev = torch.device("cuda:0")
    pair, prm, desc, bits = workload(args.workload)
    prm = dict(prm, storage=args.storage)
    h, w = pair.frame0.shape
    f0 = torch.from_numpy(pair.frame0).to(dev)
    f1 = torch.from_numpy(pair.frame1).to(dev)
    out = torch.empty((2, h, w), dtype=torch.float32, device=dev)
    handle = ofv.Handle(w, h, 1)
    if args.variant == "tuned":
        handle.autotune(f0, f1, prm, bit_depth=bits, repeats=3)
    else:
        handle.set_gn_variant(args.variant)

    def step():
        ofv.compute_flow(f0, f1, prm, bit_depth=bits, out=out, handle=handle)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    eager_ref = out.clone()

    graph = None
    if not args.no_graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step()
        torch.cuda.current_stream().wait_stream(s)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        handle.bind_stream()
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        if not torch.equal(out, eager_ref):
            raise RuntimeError("graph replay differs from the eager result")

    run = graph.replay if graph is not None else step
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if not torch.equal(out, eager_ref):
        raise RuntimeError("timed steps changed the result")
    sec = (t1 - t0) / args.steps
    mvec = w * h / sec / 1e6

    # ---- dominant kernel: Gauss-Newton iteration at full resolution, same
    # launch configuration as inside the pipeline, timed with HIP events on
    # the stream it is launched on (torch's current stream, bound to the handle).
    kr = prm["kernel_radius"]
    p0 = ofv.stage_normalize(f0, prm["norm_radius"], prm["norm_eps"], args.storage, bit_depth=bits, handle=handle)
    p1 = ofv.stage_normalize(f1, prm["norm_radius"], prm["norm_eps"], args.storage, bit_depth=bits, handle=handle)
    fin = out.clone()
    for _ in range(10):
        ofv.stage_gn_iteration(p0, p1, fin, "direct", kr, prm["reg_rel"], prm["reg_abs"], handle=handle)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.kernel_launches):
        ofv.stage_gn_iteration(p0, p1, fin, "direct", kr, prm["reg_rel"], prm["reg_abs"], handle=handle)
    ev1.record()
    torch.cuda.synchronize()
    kern_s = ev0.elapsed_time(ev1) / 1e3 / args.kernel_launches
    s_bytes = 4 if args.storage == "f32" else 2
    bytes_per_px = 2 * s_bytes + 16            # P0, P1, V in, V out
    algo_bytes = bytes_per_px * w * h
    achieved = algo_bytes / kern_s / 1e9

    # whole-step algorithmic bytes (per-sweep model) for context
    L, it = prm["num_levels"], prm["iterations"]
    in_bytes = {8: 1, 12: 2, 16: 2}.get(bits, 4)
    lw, lh = [w], [h]
    for _ in range(L - 1):
        lw.append((lw[-1] + 1) // 2)
        lh.append((lh[-1] + 1) // 2)
    npx = [a * b for a, b in zip(lw, lh)]
    step_bytes = 2 * in_bytes * npx[0] + 2 * s_bytes * npx[0]
    step_bytes += sum(2 * s_bytes * (npx[l - 1] + npx[l]) for l in range(1, L))
    for l in range(L):
        first = (2 * s_bytes + 10) if l < L - 1 else (2 * s_bytes + 8)
        step_bytes += npx[l] * (first + (it - 1) * (2 * s_bytes + 16))

    result = {
        "metric": "dense-flow Mvectors/s (fields/s at 1/4/21 Mp), % HBM roofline, bwd/fwd time",
        "value": round(mvec, 2),
        "unit": "Mvectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else f"{args.storage}-storage/f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "height": h, "width": w,
                   "num_levels": L, "kernel_radius": kr, "iterations": it,
                   "norm_radius": prm["norm_radius"], "storage": args.storage,
                   "pairs_per_step": 1, "launch": "hipGraph replay" if graph is not None else "eager",
                   "gn_decomposition": args.variant,
                   "tuning_table": handle.tuning_table().strip().splitlines() if args.variant == "tuned" else []},
        "fields_per_s": round(1.0 / sec, 1),
        "step_algorithmic_GBps": round(step_bytes / sec / 1e9, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": f"gn_kernel<{kr},{args.storage}> full resolution {w}x{h}",
                     "bytes_per_launch": algo_bytes, "us_per_launch": round(kern_s * 1e6, 3)},
    }

    if not args.no_cpu_baseline:
        import oracle
        nthreads = torch.get_num_threads()
        runs, t_cpu = 0, 0.0
        while t_cpu < args.cpu_seconds and runs < 20:
            tc = time.perf_counter()
            oracle.compute_flow(pair.frame0, pair.frame1, prm, bit_depth0=bits)
            t_cpu += time.perf_counter() - tc
            runs += 1
        result["cpu_baseline"] = {"value": round(runs * w * h / t_cpu / 1e6, 4), "unit": "Mvectors/s",
                                  "cores": nthreads, "kind": "oracle",
                                  "sample": f"{runs} run(s) of the FP64 oracle on the same {w}x{h} pair "
                                            f"({t_cpu:.1f} s)"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
