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
# Non-packed FP32/integer VALU issue rate of the chip: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz (a wave64 VALU instruction holds a 16-lane SIMD for 4 cycles;
# packed-FP32 instructions, which would double it, are not used).
VALU_LANE_INSTR_PER_S = 256 * 4 * 16 * 2.4e9
GN_NAMES = {0: "march", 1: "tile64x32", 2: "tile64x16", 3: "tile32x16", 4: "tile16x16", 5: "tile64x32w",
            6: "tile64x16w", 7: "tile64x64", 8: "tile16x16w", 9: "tile32x16w", 10: "tile32x32w", 11: "band"}
GN_SOURCES = ["ofv_gn_impl.h", "ofv_gn_tile.h", "ofv_gn_band.h", "ofv_px.h", "ofv_internal.h"]


def host_cpu():
    """Model name of the host CPU and its logical core count."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return f"{name}, {os.cpu_count()} logical cores"


def gn_source_digest():
    """sha256 over the sources of the Gauss-Newton kernels (a traffic figure is valid for one digest only)."""
    import hashlib
    hsh = hashlib.sha256()
    for f in GN_SOURCES:
        with open(os.path.join(ROOT, "paper_2509_25924_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()[:16]


def measured_traffic(workload, storage, decomposition, kind="traffic"):
    """HBM bytes (kind "traffic") or VALU instructions (kind "valu") per launch of the full-resolution
    Gauss-Newton kernel, from the committed hardware-counter summary, or None when there is none for these
    kernel sources."""
    path = os.path.join(ROOT, "profiles", f"gn_{kind}_{workload}_{storage}.md")
    if not os.path.exists(path):
        return None
    digest, table = None, {}
    for line in open(path):
        parts = line.strip().strip("|").split("|")
        if line.startswith("source digest:"):
            digest = line.split(":", 1)[1].strip()
        elif len(parts) >= 4 and parts[0].strip() in GN_NAMES.values():
            try:
                table[parts[0].strip()] = int(parts[-1].strip())
            except ValueError:
                pass
    if digest != gn_source_digest():
        return None
    return table.get(decomposition)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="shear_1mp", choices=["shear_1mp", "rankine_256", "paper_1mp", "wake_21mp"],
                    help="wake_21mp (5120x4096 cylinder wake, KR 10) only with --pmc-probe")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of replaying a hipGraph")
    ap.add_argument("--variant", default="tuned", choices=["tuned", "auto"] + list(GN_NAMES.values()),
                    help="Gauss-Newton work decomposition: autotuned per level (default) or forced")
    ap.add_argument("--tuning-table", default=None,
                    help="with --variant tuned: load this decomposition table (ofv tuning-table text) instead of "
                         "autotuning, e.g. to run a profiled command with the decompositions of an unprofiled one")
    ap.add_argument("--save-tuning", default=None, help="write the decomposition table the run used to this file")
    ap.add_argument("--kernel-launches", type=int, default=200, help="launches timed for the dominant kernel")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-21mp", action="store_true",
                    help="skip the roofline of the 5120x4096 level-0 Gauss-Newton launch (above the Infinity Cache)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="for hardware-counter runs: launch a 256 MiB elementwise negation and a 256 MiB copy 3 times each, then the full-resolution "
                         "Gauss-Newton kernel 5 times in each decomposition, and exit")
    ap.add_argument("--sweep-realisations", type=int, default=10,
                    help="particle fields per image of the accuracy sweep (the paper uses 10)")
    ap.add_argument("--suite", default=None,
                    choices=["batch4mp", "live21mp", "stream21mp", "sweep", "estimators", "adjoint512", "paper",
                             "oracle", "preprocess", "livestep", "all"],
                    help="run an additional measurement instead of the default workload (one JSON line each)")
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


# ---------------------------------------------------------------------------
# Additional measurements (one JSON line each): batched reduced-precision
# 4 Mp pairs, the 21 Mp live loop with uneven batches, the adjoint's cost, and
# the paper's own throughput setting.
# ---------------------------------------------------------------------------

def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _sweep_bytes(levels, w, h, iters, s_bytes, in_bytes, npairs=1):
    lw, lh = [w], [h]
    for _ in range(levels - 1):
        lw.append((lw[-1] + 1) // 2)
        lh.append((lh[-1] + 1) // 2)
    npx = [a * b for a, b in zip(lw, lh)]
    b = 2 * in_bytes * npx[0] + 2 * s_bytes * npx[0]
    b += sum(2 * s_bytes * (npx[l - 1] + npx[l]) for l in range(1, levels))
    for l in range(levels):
        first = (2 * s_bytes + 10) if l < levels - 1 else (2 * s_bytes + 8)
        b += npx[l] * (first + (iters - 1) * (2 * s_bytes + 16))
    return b * npairs


def _step_models(per_sweep, fused, sec):
    """A whole step's bytes over its time under both algorithmic models, as fractions of HBM peak:
    per_sweep (_sweep_bytes: every iteration streams its level's planes and field) and fused_iterations
    (the bound if all iterations of a level ran on chip: the first iteration's traffic only, i.e.
    _sweep_bytes with one iteration)."""
    return {m: {"bytes": int(b), "GBps": round(b / sec / 1e9, 1), "frac_of_8TBps": round(b / sec / 8e12, 4)}
            for m, b in (("per_sweep", per_sweep), ("fused_iterations", fused))}


def suite_batch4mp(args, dev):
    """64 time-resolved 2048x2048 12-bit turbulence pairs in one call, FP16 storage."""
    import torch
    import paper_2509_25924_amd as ofv
    import synth
    from synth.gpu_render import make_pair_device
    n_distinct, n = 8, 64
    f0s, f1s, gts = [], [], {}
    checked = (0, 21, 42, 63)                      # pairs whose accuracy is measured against the oracle
    for t in range(n_distinct):
        flow = synth.Turbulence(seed=3, rms=2.0, dmax_cap=8.0, ref_h=256, ref_w=256, t=float(t))
        want_gt = any(c % n_distinct == t for c in checked)
        a, b, gt = make_pair_device(2048, 2048, flow, fwhm=2.5, ppp=0.1, seed=3000 + t, bit_depth=12,
                                    noise=0.01 * 4095, device=dev, max_disp=8.0, with_gt=want_gt)
        gts[t] = gt
        f0s.append(a)
        f1s.append(b)
    f0s = [f0s[i % n_distinct] for i in range(n)]
    f1s = [f1s[i % n_distinct] for i in range(n)]
    prm = {"num_levels": 5, "kernel_radius": 4, "iterations": 3, "norm_radius": 2}
    outs = [torch.empty((2, 2048, 2048), dtype=torch.float32, device=dev) for _ in range(n)]
    hb = ofv.Handle(2048, 2048, n)
    res = {}
    for storage in ("f16", "f32"):
        for variant in ("auto", "tile64x16", "tile64x32", "tile64x16w", "tile64x32w", "march"):
            hb.set_gn_variant(variant)
            p = dict(prm, storage=storage)
            sec = _timed(lambda: ofv.compute_flow_batch(f0s, f1s, p, bit_depth=12, outs=outs, handle=hb), 3, 1)
            res[f"{storage}/{variant}"] = sec
    # the batch autotuner: every decomposition per level and flow mode, timed on this batch
    hb.set_gn_variant("auto")
    for storage in ("f16", "f32"):
        p = dict(prm, storage=storage)
        hb.autotune_batch(f0s, f1s, p, bit_depth=12, repeats=2)
        res[f"{storage}/tuned"] = _timed(lambda: ofv.compute_flow_batch(f0s, f1s, p, bit_depth=12, outs=outs,
                                                                        handle=hb), 3, 1)
    best = min((v, k) for k, v in res.items() if k.startswith("f16"))
    # accuracy of pairs 0, 21, 42 and 63 in FP16 and FP32 against the FP64 oracle and the ground truth;
    # the floor is the FP64 oracle with its image planes rounded to FP16 (the error that FP16 storage
    # causes by itself); "converged" pixels are those where the oracle's own endpoint error against the
    # ground truth is at most 1 px
    import numpy as np
    import oracle
    hb.set_gn_variant("auto")
    bnd = 4 * 2 ** 4
    inner = (slice(None), slice(bnd, -bnd), slice(bnd, -bnd))
    acc = {}
    for c in checked:
        gt0 = gts[c % n_distinct]
        fr0 = f0s[c].cpu().numpy().astype(np.uint16)
        fr1 = f1s[c].cpu().numpy().astype(np.uint16)
        vor = oracle.compute_flow(fr0, fr1, prm, bit_depth0=12).numpy()
        v_floor = oracle.compute_flow(fr0, fr1, prm, bit_depth0=12, plane_round="f16").numpy()
        rms_orc = float(np.sqrt(np.mean((vor - gt0)[inner] ** 2)))
        conv = np.sqrt(((vor - gt0) ** 2).sum(0)) <= 1.0

        def stats(v, tol):
            d = np.abs(v - vor).max(axis=0)
            rms = float(np.sqrt(np.mean((v - gt0)[inner] ** 2)))
            return {"max_abs_vs_oracle_px": round(float(d.max()), 5),
                    "max_abs_converged_px": round(float(d[conv].max()), 5),
                    "p99_99_abs_vs_oracle_px": round(float(np.quantile(d, 0.9999)), 6),
                    f"frac_over_{tol:g}": float(np.mean(d > tol)),
                    f"frac_over_{tol:g}_converged": float(np.mean(d[conv] > tol)),
                    "rms_vs_gt_px": round(rms, 5), "rms_ratio_vs_oracle": round(rms / rms_orc, 4)}

        row = {"rms_vs_gt_oracle_px": round(rms_orc, 5), "frac_converged": float(conv.mean()),
               "floor_f16_planes": stats(v_floor, 2e-2)}
        for st, tol in (("f16", 2e-2), ("f32", 1e-3)):
            v = ofv.compute_flow_batch(f0s[c:c + 1], f1s[c:c + 1], dict(prm, storage=st), bit_depth=12, handle=hb)[0]
            row[st] = stats(v.cpu().double().numpy(), tol)
        acc[f"pair{c}"] = row
    # the plain FP32 single-pair path on the same pairs
    h1 = ofv.Handle(2048, 2048, 1)
    h1.autotune(f0s[0], f1s[0], dict(prm, storage="f32"), bit_depth=12, repeats=2)
    out1 = outs[0]
    sec1 = _timed(lambda: [ofv.compute_flow(f0s[i], f1s[i], dict(prm, storage="f32"), bit_depth=12, out=out1,
                                            handle=h1) for i in range(n)], 2, 1)
    byts = _sweep_bytes(5, 2048, 2048, 3, 2, 2, n)
    return {"metric": "batched fields/s (64 x 2048x2048, FP16 storage)", "value": round(n / best[0], 1),
            "unit": "fields/s", "mvectors_per_s": round(n * 2048 * 2048 / best[0] / 1e6, 1),
            "decomposition": best[1], "seconds_per_batch": {k: round(v, 5) for k, v in res.items()},
            "fp32_single_pair_fields_per_s": round(n / sec1, 1),
            "speedup_vs_fp32_single_pair": round(sec1 / best[0], 2),
            "step_algorithmic_GBps": round(byts / best[0] / 1e9, 1),
            "step_bytes_models": _step_models(byts, _sweep_bytes(5, 2048, 2048, 1, 2, 2, n), best[0]), "accuracy": acc,
            "data": "synthetic: 8 distinct time steps of a 256-mode k^-5/3 field tiled to 64 pairs"}


def suite_live21mp(args, dev):
    """21 Mp cylinder-wake frames, uneven batch {5120x4096, 2048^2 crop, 1024^2 crop} per step, hipGraph loop;
    compute-only and streaming (one new 12-bit frame per step uploaded from a pinned host ring while the
    previous step computes)."""
    import numpy as np
    import torch
    import paper_2509_25924_amd as ofv
    import oracle
    import synth
    from synth.gpu_render import make_pair_device
    W, H = 5120, 4096
    phases = 16
    pairs, gt0 = [], None
    for ph in range(phases):
        flow = synth.CylinderWake(H, W, t=200.0 * ph / phases, dmax=10.0)
        a, b, gt = make_pair_device(H, W, flow, fwhm=2.5, ppp=0.1, seed=4000 + ph, bit_depth=12,
                                    noise=0.01 * 4095, device=dev, max_disp=10.0, with_gt=(ph == 0))
        pairs.append((a, b))
        gt0 = gt if ph == 0 else gt0
    prm = {"num_levels": 4, "kernel_radius": 10, "iterations": 3, "norm_radius": 2}
    hb = ofv.Handle(W, H, 3)
    outs = [torch.empty((2, H, W), dtype=torch.float32, device=dev),
            torch.empty((2, 2048, 2048), dtype=torch.float32, device=dev),
            torch.empty((2, 1024, 1024), dtype=torch.float32, device=dev)]
    crop2 = (slice(1024, 3072), slice(1536, 3584))
    crop1 = (slice(1536, 2560), slice(2048, 3072))

    hdef = ofv.Handle(W, H, 3)      # no tuned table: the default decomposition choice
    cur = [hb]

    def batch_of(a, b, p):
        f0 = [a, a[crop2], a[crop1]]
        f1 = [b, b[crop2], b[crop1]]
        ofv.compute_flow_batch(f0, f1, p, bit_depth=12, outs=outs, handle=cur[0])

    def capture(fn):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn()
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        cur[0].bind_stream()
        return g

    res, acc, tables = {}, {}, {}
    steps = 500
    for storage in ("bf16", "f32"):
        p = dict(prm, storage=storage)
        # the autotuner on the uneven batch itself: per launch group (level, flow mode) the fastest
        # decomposition, keyed by the batch's geometry
        hb.set_gn_variant("auto")
        a0, b0 = pairs[0]
        hb.autotune_batch([a0, a0[crop2], a0[crop1]], [b0, b0[crop2], b0[crop1]], p, bit_depth=12, repeats=3)
        tables[storage] = [l for l in hb.tuning_table().splitlines() if l.split()[1] == str({"f32": 0, "bf16": 2}[storage])]
        for variant in ("tuned", "default"):
            cur[0] = hb if variant == "tuned" else hdef
            graphs = [capture(lambda ph=ph: batch_of(*pairs[ph], p)) for ph in range(phases)]
            k = [0]

            def step():
                graphs[k[0] % phases].replay()
                k[0] += 1
            res[f"{storage}/{variant}"] = _timed(step, steps, 16)
            del graphs
        # accuracy of the 1024^2 crop of phase 0 against the FP64 oracle (tuned decompositions)
        cur[0] = hb
        batch_of(*pairs[0], p)
        v = outs[2].cpu().double().numpy()
        a0 = pairs[0][0][crop1].cpu().numpy().astype(np.uint16)
        b0 = pairs[0][1][crop1].cpu().numpy().astype(np.uint16)
        ref = oracle.compute_flow(a0, b0, prm, bit_depth0=12).numpy()
        d = np.abs(v - ref).max(axis=0)
        g = gt0[(slice(None),) + crop1]
        rms = lambda x: float(np.sqrt(np.mean((x - g)[:, 80:-80, 80:-80] ** 2)))
        acc[storage] = {"max_abs_vs_oracle_px": round(float(d.max()), 5),
                        "p99_99_abs_vs_oracle_px": round(float(np.quantile(d, 0.9999)), 6),
                        "frac_over_1e-3": float(np.mean(d > 1e-3)), "frac_over_2e-2": float(np.mean(d > 2e-2)),
                        "rms_vs_gt_px": round(rms(v), 5), "rms_vs_gt_oracle_px": round(rms(ref), 5)}
    best_key = min(res, key=res.get)
    best = res[best_key]
    per = {k: round(1.0 / v, 1) for k, v in res.items()}
    vec = W * H + 2048 * 2048 + 1024 * 1024

    # streaming: frame j of the sequence is phase j's frame 0; step k computes the pair (frame k,
    # frame k+1) from a ring of three device frames while frame k+2 is copied in on a second stream
    storage, variant = best_key.split("/")
    p = dict(prm, storage=storage)
    cur[0] = hb if variant == "tuned" else hdef

    # the paper's live criterion: frames arrive at a fixed rate, raised until overruns appear (a frame
    # whose field is not complete when the next frame arrives); compute-only graph steps, host clock
    from paper_2509_25924_amd.live import LiveLoop, max_overrun_free_rate
    ograph = [capture(lambda ph=ph: batch_of(*pairs[ph], p)) for ph in range(phases)]
    overrun = max_overrun_free_rate(
        lambda period: LiveLoop(lambda k: ograph[k % phases].replay(), period, wait=torch.cuda.synchronize),
        [90.0, 200.0, 300.0, 350.0, 400.0, 450.0, 500.0, 600.0, 650.0, 700.0], 200)
    del ograph
    nhost = 4
    host = [torch.empty((H, W), dtype=torch.int16, pin_memory=True) for _ in range(nhost)]
    for j in range(nhost):
        host[j].copy_(pairs[j][0])
    ring = [torch.empty((H, W), dtype=torch.int16, device=dev) for _ in range(3)]
    for j in range(2):
        ring[j].copy_(host[j])
    graphs = [capture(lambda r=r: batch_of(ring[r], ring[(r + 1) % 3], p)) for r in range(3)]
    copy_stream = torch.cuda.Stream()
    comp = torch.cuda.current_stream()
    done = [torch.cuda.Event() for _ in range(3)]      # compute that last read ring slot r has finished
    ready = [torch.cuda.Event() for _ in range(3)]     # ring slot r holds its frame
    for r in range(3):
        done[r].record(comp)
        ready[r].record(comp)
    ks = [0]

    def stream_step():
        k = ks[0]
        nxt = (k + 2) % 3
        with torch.cuda.stream(copy_stream):
            copy_stream.wait_event(done[nxt])
            ring[nxt].copy_(host[(k + 2) % nhost], non_blocking=True)
            ready[nxt].record(copy_stream)
        comp.wait_event(ready[k % 3])
        comp.wait_event(ready[(k + 1) % 3])
        graphs[k % 3].replay()
        done[k % 3].record(comp)
        done[(k + 1) % 3].record(comp)
        ks[0] += 1
    sec_stream = _timed(stream_step, steps, 16)
    t0 = time.perf_counter()
    for _ in range(20):
        ring[0].copy_(host[0], non_blocking=True)
    torch.cuda.synchronize()
    h2d = 20 * ring[0].numel() * 2 / (time.perf_counter() - t0) / 1e9
    sb = 2 if best_key.startswith("bf16") else 4      # planes of the fastest configuration
    byts, byts_fused = (sum(_sweep_bytes(4, sw, sh, its, sb, 2) for sw, sh in ((W, H), (2048, 2048), (1024, 1024)))
                        for its in (3, 1))

    # live derived quantities of the 21 Mp field in every step (vorticity plane, recirculation area
    # outside the cylinder, 64 probes along the wake centre line), captured in the same graph
    yy, xx = torch.meshgrid(torch.arange(H, device=dev), torch.arange(W, device=dev), indexing="ij")
    dmask = (((xx - 1024.0) ** 2 + (yy - 2048.0) ** 2) > 200.0 ** 2).to(torch.uint8)
    del yy, xx
    dprobes = torch.stack([torch.linspace(1300.0, 5000.0, 64), torch.full((64,), 2048.0)], 1).to(dev)
    dkw = dict(mask=dmask, dx=1e-4, dz=1e-4, dt=0.01, probes=dprobes, handle=hb)   # 0.1 mm pixels, 100 Hz
    held = {}

    def batch_derived(a, b, p, ph):
        batch_of(a, b, p)
        held[ph] = ofv.derived(outs[0], **dkw)
    graphs = [capture(lambda ph=ph: batch_derived(*pairs[ph], p, ph)) for ph in range(phases)]
    k = [0]

    def dstep():
        graphs[k[0] % phases].replay()
        k[0] += 1
    sec_derived = _timed(dstep, steps, 16)
    torch.cuda.synchronize()
    eager = ofv.derived(outs[0], **dkw)
    torch.cuda.synchronize()
    last = held[(k[0] - 1) % phases]    # outputs of the graph replayed last
    if not (torch.equal(eager["vorticity"], last["vorticity"]) and torch.equal(eager["area"], last["area"])
            and torch.equal(eager["probes"], last["probes"])):
        raise RuntimeError("derived quantities of the graph replay differ from an eager call")
    del graphs
    nrep = 50
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(nrep):
            ofv.derived(outs[0], **dkw)
    hb.bind_stream()
    g.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    d_us = e0.elapsed_time(e1) * 1e3 / nrep
    del g
    d_bytes = (8 + 1 + 4) * W * H          # flow in, mask in, vorticity out
    # two streams (measured last: the streams it adds change how later streams map onto the hardware
    # queues): consecutive steps alternate between two handles (the best configuration's table), so
    # that one step's preprocessing and coarse levels overlap the other's large launches
    hb2 = ofv.Handle(W, H, 3)
    if variant == "tuned":
        hb2.load_tuning_table(hb.tuning_table())
    outs_b = [outs, [torch.empty_like(o) for o in outs]]

    def make_live_step(hd, i):
        def one(ph):
            a, b = pairs[ph]
            ofv.compute_flow_batch([a, a[crop2], a[crop1]], [b, b[crop2], b[crop1]], p, bit_depth=12,
                                   outs=outs_b[i], handle=hd)
        return [lambda ph=ph: one(ph) for ph in range(0, phases, 2)]
    sec_two = time_two_streams(make_live_step, [cur[0], hb2], steps, 16)
    hb2.close()
    cur[0].bind_stream()

    derived_info = {"steps_per_s_with_derived": round(1.0 / sec_derived, 1),
                    "kernel_us_5120x4096": round(d_us, 2), "bytes_per_call": d_bytes,
                    "algorithmic_GBps": round(d_bytes / d_us / 1e3, 1),
                    "frac_of_8TBps": round(d_bytes / d_us / 1e3 / HBM_PEAK_GBS, 4),
                    "outputs": "vorticity plane, recirculation area (pixels outside the cylinder), 64 probes",
                    "recirculation_area_cm2": round(float(eager["area"].item()) * 1e4, 3)}
    return {"metric": "live steps/s (5120x4096 + 2048^2 + 1024^2 uneven batch per step, hipGraph)",
            "value": round(1.0 / best, 1), "unit": "steps/s", "steps": steps, "best": best_key,
            "tuning_table": tables,
            "overrun_sweep": overrun,
            "gvectors_per_s": round(vec / best / 1e9, 3), "steps_per_s_by_config": per,
            "fields_per_s_each_size": round(1.0 / best, 1),
            "step_algorithmic_GBps": round(byts / best / 1e9, 1),
            "step_bytes_models": _step_models(byts, byts_fused, best),
            "streaming_steps_per_s": round(1.0 / sec_stream, 1),
            "two_stream_steps_per_s": round(1.0 / sec_two, 1),
            "streaming": "one new 12-bit 5120x4096 frame (42 MB) per step, pinned host ring -> 3 device slots, "
                         "copy stream overlapped with the graph replay",
            "h2d_GBps_pinned": round(h2d, 1),
            "derived": derived_info,
            "accuracy_1024_crop": acc,
            "data": "synthetic: 16 phases of a cylinder wake (potential flow + Lamb-Oseen street, max 10 px)"}


def suite_stream21mp(args, dev):
    """A time-resolved 5120x4096 sequence (16 frames of a cylinder wake, cycled): pair calls that normalise
    and reduce both frames of every pair, against pushes that normalise and reduce each new frame once
    and pair it with the retained pyramid of the previous one; both as hipGraph loops, the live
    configuration's parameters (L 4, KR 10, IT 3, NR 2, FP32 storage)."""
    import torch
    import paper_2509_25924_amd as ofv
    import synth
    from synth.gpu_render import make_pair_device
    W, H = 5120, 4096
    nf = 16
    seq = []
    for ph in range(nf):
        flow = synth.CylinderWake(H, W, t=200.0 * ph / nf, dmax=10.0)
        a, _, _ = make_pair_device(H, W, flow, fwhm=2.5, ppp=0.1, seed=4000 + ph, bit_depth=12,
                                   noise=0.01 * 4095, device=dev, max_disp=10.0, with_gt=False)
        seq.append(a)
    prm = {"num_levels": 4, "kernel_radius": 10, "iterations": 3, "norm_radius": 2}
    h = ofv.Handle(W, H, 1)
    out = torch.empty((2, H, W), dtype=torch.float32, device=dev)

    def capture(fn):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn()
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        h.bind_stream()
        return g

    steps = 200
    # pair calls: step k computes (frame k-1, frame k)
    graphs = [capture(lambda k=k: ofv.compute_flow(seq[(k - 1) % nf], seq[k], prm, bit_depth=12, out=out,
                                                   handle=h)) for k in range(nf)]
    kk = [1]

    def pair_step():
        graphs[kk[0] % nf].replay()
        kk[0] += 1
    sec_pair = _timed(pair_step, steps, 16)
    torch.cuda.synchronize()
    ref = out.clone()                                   # pair (frame k-1, frame k) of the last replay
    last_k = (kk[0] - 1) % nf
    del graphs
    # pushes: frame k goes to slab k % 2 (nf is even, so the slab of a frame never changes)
    h.stream_reset()
    h.stream_push(seq[0], prm, bit_depth=12, out=out)
    pushes = {}
    for k in list(range(1, nf)) + [0]:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            h.stream_push(seq[k], prm, bit_depth=12, out=out)
        pushes[k] = g
    h.bind_stream()
    h.stream_reset()
    h.stream_push(seq[0], prm, bit_depth=12, out=out)   # retained frame 0 in slab 0, as at capture
    ks = [1]

    def push_step():
        pushes[ks[0] % nf].replay()
        ks[0] += 1
    # the replays must continue the sequence from frame 1: warm-up and timed steps run in order
    sec_push = _timed(push_step, steps, 16)
    torch.cuda.synchronize()
    # the push loop ends on frame (ks - 1); recompute the pair check for the same frames
    lk = (ks[0] - 1) % nf
    chk = ofv.compute_flow(seq[(lk - 1) % nf], seq[lk], prm, bit_depth=12, handle=ofv.Handle(W, H, 1))
    torch.cuda.synchronize()
    if not torch.equal(chk, out):
        raise RuntimeError("streamed field differs from the pair call on the same frames")
    del pushes
    return {"metric": "time-resolved 5120x4096 sequence: steps/s with each frame reduced once (stream push) vs "
                      "pair calls", "value": round(1.0 / sec_push, 1), "unit": "steps/s", "steps": steps,
            "pair_calls_steps_per_s": round(1.0 / sec_pair, 1), "speedup": round(sec_pair / sec_push, 3),
            "ms_per_step_stream": round(sec_push * 1e3, 3), "ms_per_step_pairs": round(sec_pair * 1e3, 3),
            "checked": f"streamed field of frames ({(lk - 1) % nf}, {lk}) equals the pair call bit for bit",
            "params": prm, "data": "synthetic: 16 frames of a cylinder wake (potential flow + Lamb-Oseen street)"}


def suite_sweep(args, dev):
    """The paper's accuracy study on synthetic Rankine vortices, on the batched estimator: every image of
    its Rankine grid (maximum displacement 8-32 px x 5-15 particles per 16x16 window x core radius
    12-150 px: 72 images of 1024^2, 8-bit, no noise) x every setting of its estimator grid (KR 2-7,
    PSL 2-4, IT 1-4, NR 1-4: 288), for `--sweep-realisations` particle fields; scored by Psi and <Err>;
    the setting with the lowest Psi per (core radius, displacement), compared with the paper's table."""
    import itertools
    import json as _json
    import numpy as np
    import torch
    import paper_2509_25924_amd as ofv
    import synth
    from synth import metrics as M
    from synth.gpu_render import make_pair_device
    S = 1024
    c = (S - 1) / 2.0
    nreal = args.sweep_realisations
    ig, og = M.rankine_grid(), M.ofv_grid()
    imgs = list(itertools.product(ig["dmax"], ig["part_per_iw"], ig["radius"]))
    settings = list(itertools.product(og["kernel_radius"], og["psl"], og["iterations"], og["norm_radius"]))
    fwhm = 0.75 * synth.FWHM_PER_SIGMA          # particle image diameter 3 px taken as the e^-2 diameter (4 sigma)
    vort = [synth.Rankine(c, c, float(R), float(D)) for D, _, R in imgs]
    yy, xx = np.mgrid[0:S, 0:S].astype(np.float64)
    gts = torch.stack([torch.as_tensor(np.stack(v(xx, yy)), dtype=torch.float32) for v in vort]).to(dev)
    del yy, xx
    radii = sorted(set(R for _, _, R in imgs))
    unf = {R: M.Unfolding(c, c, M.default_r_max(R, S, S), dev) for R in radii}
    groups = {R: [i for i, (_, _, r) in enumerate(imgs) if r == R] for R in radii}
    theory = {R: torch.stack([unf[R].theory(vort[i], torch.float32) for i in groups[R]]) for R in radii}
    n = len(imgs)
    hd = ofv.Handle(S, S, n)
    outs = [torch.empty((2, S, S), dtype=torch.float32, device=dev) for _ in range(n)]
    psi_sum = np.zeros((n, len(settings)))
    err_sum = np.zeros((n, len(settings)))
    est_s, t_start = 0.0, time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for rz in range(nreal):
        f0, f1 = [], []
        for i, (D, ppi, R) in enumerate(imgs):
            a, b, _ = make_pair_device(S, S, vort[i], fwhm=fwhm, ppp=ppi / 256.0, seed=7000 + 1000 * rz + i,
                                       bit_depth=8, noise=0.0, device=dev, max_disp=float(D))
            f0.append(a)
            f1.append(b)
        for si, (kr, psl, it, nr) in enumerate(settings):
            prm = {"num_levels": psl + 1, "kernel_radius": kr, "iterations": it, "norm_radius": nr}
            e0.record()
            ofv.compute_flow_batch(f0, f1, prm, bit_depth=8, outs=outs, handle=hd)
            e1.record()
            for R in radii:
                idx = groups[R]
                fl = torch.stack([outs[i] for i in idx])
                psi_sum[idx, si] += unf[R].psi(fl, theory[R]).cpu().numpy()
                err_sum[idx, si] += M.mean_endpoint_error(fl, gts[idx], 16).cpu().numpy()
            est_s += e0.elapsed_time(e1) / 1e3
        del f0, f1
    total_s = time.perf_counter() - t_start
    psi_m, err_m = psi_sum / nreal, err_sum / nreal
    paper = _json.load(open(os.path.join(ROOT, "tests", "golden", "paper_numbers.json")))["rankine_best_settings"]
    rows = []
    for R, D, ppi_p, kr_p, nr_p, psl_p, it_p in paper["rows"]:
        cand = [i for i, (d, _, r) in enumerate(imgs) if d == D and r == R]
        i, si = min(((i, int(np.argmin(psi_m[i]))) for i in cand), key=lambda t: psi_m[t[0], t[1]])
        kr, psl, it, nr = settings[si]
        rows.append({"R": R, "D": D, "D_over_R": round(D / R, 3), "particles_per_iw": imgs[i][1], "KR": kr,
                     "NR": nr, "PSL": psl, "IT": it, "psi": round(float(psi_m[i, si]), 4),
                     "mean_err_px": round(float(err_m[i, si]), 4),
                     "paper": {"particles_per_iw": ppi_p, "KR": kr_p, "NR": nr_p, "PSL": psl_p, "IT": it_p}})

    def spearman(a, b):
        rank = lambda x: np.argsort(np.argsort(np.asarray(x, float), kind="stable"), kind="stable").astype(float)
        return float(np.corrcoef(rank(a), rank(b))[0, 1])
    dr = [r["D_over_R"] for r in rows]
    ours_kr = [r["KR"] for r in rows]
    paper_kr = [r["paper"]["KR"] for r in rows]
    flows = n * len(settings) * nreal
    return {"metric": "accuracy sweep: Rankine image grid x estimator grid, fields/s of the batched estimator",
            "value": round(flows / est_s, 1), "unit": "fields/s", "fields": flows, "realisations": nreal,
            "estimator_seconds": round(est_s, 2), "wall_seconds": round(total_s, 1),
            "spearman_DR_vs_best_KR": {"ours": round(spearman(dr, ours_kr), 3),
                                        "paper": round(spearman(dr, paper_kr), 3)},
            "best_KR_equal_to_paper": int(sum(a == b for a, b in zip(ours_kr, paper_kr))),
            "best_KR_mean_abs_diff": round(float(np.mean(np.abs(np.subtract(ours_kr, paper_kr)))), 3),
            "best_psi_median": round(float(np.median([r["psi"] for r in rows])), 4),
            "best_settings": rows,
            "data": "synthetic Rankine vortices at 1024^2 (Gaussian particles of 3 px e^-2 diameter, 8-bit, no "
                    "noise, no out-of-plane loss) standing in for the paper's generator images"}


def suite_estimators(args, dev):
    """The three estimators side by side on the paper's Rankine image grid (72 images of 1024^2, 8-bit,
    no noise; `--sweep-realisations` particle fields): the symmetric estimator with its consistent
    update, the symmetric estimator with the increment-form update, and forward-additive Lucas-Kanade,
    at KR 3, 5 and 7 with PSL 3, IT 3, NR 2; scored by Psi and <Err> as in the sweep."""
    import itertools
    import numpy as np
    import torch
    import paper_2509_25924_amd as ofv
    import synth
    from synth import metrics as M
    from synth.gpu_render import make_pair_device
    S = 1024
    c = (S - 1) / 2.0
    nreal = args.sweep_realisations
    ig = M.rankine_grid()
    imgs = list(itertools.product(ig["dmax"], ig["part_per_iw"], ig["radius"]))
    fwhm = 0.75 * synth.FWHM_PER_SIGMA
    vort = [synth.Rankine(c, c, float(R), float(D)) for D, _, R in imgs]
    yy, xx = np.mgrid[0:S, 0:S].astype(np.float64)
    gts = torch.stack([torch.as_tensor(np.stack(v(xx, yy)), dtype=torch.float32) for v in vort]).to(dev)
    del yy, xx
    radii = sorted(set(R for _, _, R in imgs))
    unf = {R: M.Unfolding(c, c, M.default_r_max(R, S, S), dev) for R in radii}
    groups = {R: [i for i, (_, _, r) in enumerate(imgs) if r == R] for R in radii}
    theory = {R: torch.stack([unf[R].theory(vort[i], torch.float32) for i in groups[R]]) for R in radii}
    n = len(imgs)
    estimators = {"symmetric_consistent": {}, "symmetric_increment": {"update": "increment"},
                  "forward_additive": {"estimator": "forward_additive"}}
    krs = (3, 5, 7)
    hd = ofv.Handle(S, S, n)
    outs = [torch.empty((2, S, S), dtype=torch.float32, device=dev) for _ in range(n)]
    psi = {e: np.zeros((n, len(krs))) for e in estimators}
    err = {e: np.zeros((n, len(krs))) for e in estimators}
    for rz in range(nreal):
        f0, f1 = [], []
        for i, (D, ppi, R) in enumerate(imgs):
            a, b, _ = make_pair_device(S, S, vort[i], fwhm=fwhm, ppp=ppi / 256.0, seed=7000 + 1000 * rz + i,
                                       bit_depth=8, noise=0.0, device=dev, max_disp=float(D))
            f0.append(a)
            f1.append(b)
        for name, extra in estimators.items():
            for ki, kr in enumerate(krs):
                prm = dict({"num_levels": 4, "kernel_radius": kr, "iterations": 3, "norm_radius": 2}, **extra)
                ofv.compute_flow_batch(f0, f1, prm, bit_depth=8, outs=outs, handle=hd)
                for R in radii:
                    idx = groups[R]
                    fl = torch.stack([outs[i] for i in idx])
                    psi[name][idx, ki] += unf[R].psi(fl, theory[R]).cpu().numpy()
                    err[name][idx, ki] += M.mean_endpoint_error(fl, gts[idx], 16).cpu().numpy()
        del f0, f1
    names = list(estimators)
    stack_err = np.stack([err[e] / nreal for e in names])        # estimator x image x KR
    best = np.argmin(stack_err, axis=0)
    res = {}
    for k, e in enumerate(names):
        res[e] = {"mean_psi": round(float(np.mean(psi[e] / nreal)), 4),
                  "mean_err_px": round(float(np.mean(err[e] / nreal)), 4),
                  "median_err_px": round(float(np.median(err[e] / nreal)), 4),
                  "mean_err_px_by_KR": {str(kr): round(float(np.mean(err[e][:, ki] / nreal)), 4)
                                        for ki, kr in enumerate(krs)},
                  "lowest_err_share": round(float(np.mean(best == k)), 3)}
    return {"metric": "estimator comparison on the Rankine image grid (mean <Err> px, lower is better)",
            "value": res["symmetric_consistent"]["mean_err_px"], "unit": "px", "higher_is_better": False,
            "estimators": res, "settings": {"KR": list(krs), "PSL": 3, "IT": 3, "NR": 2},
            "images": n, "realisations": nreal,
            "data": "synthetic Rankine vortices at 1024^2 (Gaussian particles of 3 px e^-2 diameter, 8-bit, no "
                    "noise, no out-of-plane loss) standing in for the paper's generator images"}


def suite_oracle(args, dev):
    """The FP64 CPU oracle's own throughput on the host of the GPU: the 256^2 Rankine and 1024^2 shear
    configurations with every thread and with one, one 2048^2 turbulence pair and a 2048^2 crop of a
    5120x4096 cylinder-wake pair (live parameters) with every thread (a reported baseline, not a target)."""
    import numpy as np
    import torch
    import oracle
    import synth
    from synth.gpu_render import make_pair_device
    nthreads = torch.get_num_threads()
    rows = []

    def timed(name, f0, f1, prm, bits, threads, budget=20.0, max_runs=5):
        torch.set_num_threads(threads)
        runs, t = 0, 0.0
        while runs < 1 or (t < budget and runs < max_runs):
            t0 = time.perf_counter()
            oracle.compute_flow(f0, f1, prm, bit_depth0=bits)
            t += time.perf_counter() - t0
            runs += 1
        h, w = f0.shape
        rows.append({"config": name, "size": f"{w}x{h}", "threads": threads, "runs": runs,
                     "seconds_per_field": round(t / runs, 3), "mvectors_per_s": round(w * h * runs / t / 1e6, 4)})
        print(f"#   oracle {name} threads={threads}: {t / runs:.2f} s per field", file=sys.stderr, flush=True)

    pair, prm = synth.config_rankine_256()
    for th in (nthreads, 1):
        timed("rankine_256", pair.frame0, pair.frame1, prm, 8, th)
    pair, prm = synth.config_shear_1mp()
    for th in (nthreads, 1):
        timed("shear_1mp", pair.frame0, pair.frame1, prm, 12, th, budget=30.0, max_runs=3)
    pair, prm = synth.config_turbulence_4mp(0)
    timed("turbulence_4mp", pair.frame0, pair.frame1, dict(prm, storage="f32"), 12, nthreads, max_runs=1)
    W, H = 5120, 4096
    a, b, _ = make_pair_device(H, W, synth.CylinderWake(H, W, t=0.0, dmax=10.0), fwhm=2.5, ppp=0.1, seed=4000,
                               bit_depth=12, noise=0.01 * 4095, device=dev, max_disp=10.0)
    # a 2048^2 crop of the 5120x4096 frame with the live parameters (the whole frame takes minutes)
    crop = (slice(1024, 3072), slice(1536, 3584))
    timed("cylinder_21mp_crop2048", a[crop].cpu().numpy().astype(np.uint16), b[crop].cpu().numpy().astype(np.uint16),
          {"num_levels": 4, "kernel_radius": 10, "iterations": 3, "norm_radius": 2}, 12, nthreads, max_runs=1)
    torch.set_num_threads(nthreads)
    return {"metric": "FP64 CPU oracle throughput on the GPU host", "value": rows[2]["mvectors_per_s"],
            "unit": "Mvectors/s (1024^2 shear, every thread)", "rows": rows, "host": host_cpu(),
            "note": "plain float64 torch CPU operations, not tuned; a baseline, not a target"}


def suite_adjoint512(args, dev):
    """Backward/forward cost on 16 float 512x512 pairs (loss sum |V - V_gt|^2), batched: the adjoint after
    a forward that kept its iterates (the training pattern), the self-contained backward (which runs the
    forward itself), both in recompute and store-all mode, their device memory, and single-pair calls."""
    import torch
    import paper_2509_25924_amd as ofv
    import synth
    n = 16
    pairs = [synth.config_adjoint_512(i) for i in range(n)]
    prm = pairs[0][1]
    f0 = [torch.from_numpy(p.frame0).to(dev) for p, _ in pairs]
    f1 = [torch.from_numpy(p.frame1).to(dev) for p, _ in pairs]
    gt = [torch.from_numpy(p.gt.astype("float32")).to(dev) for p, _ in pairs]
    L, it = prm["num_levels"], prm["iterations"]
    h = ofv.Handle(512, 512, n)
    mem = {m: h.backward_workspace_bytes(L, it, n, store_all=(m == "store_all")) for m in ("recompute", "store_all")}
    h.reserve_backward(L, it, n, store_all=True)
    outs = [torch.empty((2, 512, 512), dtype=torch.float32, device=dev) for _ in range(n)]
    fwd = _timed(lambda: ofv.compute_flow_batch(f0, f1, prm, outs=outs, handle=h), 20, 3)
    fwd1 = _timed(lambda: [ofv.compute_flow(f0[i], f1[i], prm, out=outs[i], handle=h) for i in range(n)], 10, 2)
    grads = [(2 * (outs[i] - gt[i])).contiguous() for i in range(n)]
    res = {}
    for mode in ("recompute", "store_all"):
        mp = dict(prm, store_all=(mode == "store_all"))
        res[mode + "_self_contained"] = _timed(lambda: ofv.compute_flow_backward_batch(f0, f1, mp, grads, handle=h),
                                               10, 2)
        res[mode + "_saving_forward"] = _timed(
            lambda: ofv.compute_flow_batch(f0, f1, dict(mp, save_iterates=True), outs=outs, handle=h), 20, 3)
        # the saved iterates stay valid across backward calls on the same inputs
        res[mode + "_adjoint"] = _timed(
            lambda: ofv.compute_flow_backward_batch(f0, f1, dict(mp, saved_forward=True), grads, handle=h), 10, 2)
    bwd1 = _timed(lambda: [ofv.compute_flow_backward(f0[i], f1[i], prm, grads[i], handle=h) for i in range(n)], 5, 1)
    h.close()
    ms = {k: round(v * 1e3, 3) for k, v in res.items()}
    npx = sum((512 >> l) ** 2 for l in range(L))
    return {"metric": "bwd/fwd time ratio (16 x 512x512 float pairs, batched adjoint after a saving forward, "
                      "recompute mode, against the batched forward)",
            "value": round(res["recompute_adjoint"] / fwd, 2), "unit": "ratio",
            "self_contained_bwd_over_fwd": round(res["recompute_self_contained"] / fwd, 2),
            "self_contained_bwd_over_16_single_forwards": round(res["recompute_self_contained"] / fwd1, 2),
            "forward_ms_batch": round(fwd * 1e3, 3), "forward_ms_16_single": round(fwd1 * 1e3, 3),
            "backward_ms": ms, "backward_ms_16_single_self_contained": round(bwd1 * 1e3, 3),
            "store_all_over_recompute_adjoint_time": round(res["store_all_adjoint"] / res["recompute_adjoint"], 3),
            "workspace_bytes_recompute": mem["recompute"], "workspace_bytes_store_all": mem["store_all"],
            "stored_bytes_per_level_pixel_per_iteration": {"recompute": 8, "store_all": 40},
            "pixels_per_pair_all_levels": npx,
            "data": "synthetic Rankine / turbulence float frames"}


def suite_paper(args, dev):
    """The paper's throughput setting: 8-bit pairs, NR 2, KR 10, IT 3, PSL 0..2, sizes 1, 4 and 21 Mp."""
    import torch
    import paper_2509_25924_amd as ofv
    import synth
    from synth.gpu_render import make_pair_device
    rows = []
    for (w, h) in ((1024, 1024), (2048, 2048), (5120, 4096)):
        pairs = []
        for i in range(10 if w * h <= 4 << 20 else 4):
            flow = synth.Translation(1.3, -0.7, shear=0.002, y_ref=h / 2)
            pairs.append(make_pair_device(h, w, flow, fwhm=2.5, ppp=0.1, seed=5000 + i, bit_depth=8, noise=2.0,
                                          device=dev, max_disp=3.0)[:2])
        hd = ofv.Handle(w, h, 1)
        out = torch.empty((2, h, w), dtype=torch.float32, device=dev)
        for levels in (1, 2, 3):
            for storage in ("f32", "bf16"):
                prm = {"num_levels": levels, "kernel_radius": 10, "iterations": 3, "norm_radius": 2,
                       "storage": storage}
                hd.autotune(pairs[0][0], pairs[0][1], prm, bit_depth=8, repeats=2)
                k = [0]

                def one():
                    a, b = pairs[k[0] % len(pairs)]
                    ofv.compute_flow(a, b, prm, bit_depth=8, out=out, handle=hd)
                    k[0] += 1
                sec = _timed(one, 40 if w * h > 4 << 20 else 200, 5)
                byts = _sweep_bytes(levels, w, h, 3, 4 if storage == "f32" else 2, 1)
                fused = _sweep_bytes(levels, w, h, 1, 4 if storage == "f32" else 2, 1)
                rows.append({"size": f"{w}x{h}", "psl": levels - 1, "storage": storage,
                             "fields_per_s": round(1.0 / sec, 1), "mvectors_per_s": round(w * h / sec / 1e6, 1),
                             "algorithmic_GBps": round(byts / sec / 1e9, 1),
                             "frac_of_8TBps": round(byts / sec / 8e12, 4),
                             "frac_of_8TBps_fused_iterations": round(fused / sec / 8e12, 4)})
        hd.close()
    return {"metric": "fields/s at the paper's throughput setting (NR 2, KR 10, IT 3)", "rows": rows,
            "paper_rtx5090_offline_fields_per_s": {"1Mp": [1100, 1800], "4Mp": [400, 500], "21Mp": [80, 99]},
            "data": "synthetic 8-bit particle pairs (translation + shear), pre-loaded in device memory"}


def suite_livestep(args, dev):
    """One live step's launches for a kernel trace: the 5120x4096 frame with its 2048^2 and 1024^2 crops as
    one uneven batch (L 4, KR 10, IT 3, NR 2, FP32 planes, default decompositions), captured in a hipGraph
    and replayed 30 times after 5 warm-up replays."""
    import torch
    import paper_2509_25924_amd as ofv
    import synth
    from synth.gpu_render import make_pair_device
    W, H = 5120, 4096
    flow = synth.CylinderWake(H, W, t=0.0, dmax=10.0)
    a, b, _ = make_pair_device(H, W, flow, fwhm=2.5, ppp=0.1, seed=4000, bit_depth=12, noise=0.01 * 4095,
                               device=dev, max_disp=10.0, with_gt=False)
    prm = {"num_levels": 4, "kernel_radius": 10, "iterations": 3, "norm_radius": 2, "storage": "f32"}
    hb = ofv.Handle(W, H, 3)
    outs = [torch.empty((2, H, W), device=dev), torch.empty((2, 2048, 2048), device=dev),
            torch.empty((2, 1024, 1024), device=dev)]
    c2 = (slice(1024, 3072), slice(1536, 3584))
    c1 = (slice(1536, 2560), slice(2048, 3072))

    def step():
        ofv.compute_flow_batch([a, a[c2], a[c1]], [b, b[c2], b[c1]], prm, bit_depth=12, outs=outs, handle=hb)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    hb.bind_stream()
    for _ in range(5):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(30):
        g.replay()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / 30
    del g
    hb.close()
    return {"metric": "live step (5120x4096 + 2048^2 + 1024^2 uneven batch, FP32, default decompositions)",
            "value": round(1.0 / sec, 1), "unit": "steps/s", "steps": 30, "data": "synthetic cylinder-wake pair"}


def suite_preprocess(args, dev):
    """Normalisation (NR 1, 12-bit input, FP32 planes) and the three-level pyramid of one frame at 1, 4 and
    21 Mp through the stage entry points.  Host-timed averages over back-to-back calls: at 1 Mp the Python
    call rate bounds them, so the kernel durations come from a kernel trace of this suite."""
    import torch
    import paper_2509_25924_amd as ofv
    rows = []
    g = torch.Generator(device=dev).manual_seed(7)
    for (w, h) in ((1024, 1024), (2048, 2048), (5120, 4096)):
        frame = torch.randint(0, 4096, (h, w), dtype=torch.int32, device=dev, generator=g).to(torch.uint16)
        hd = ofv.Handle(w, h, 1)
        plane = ofv.stage_normalize(frame, 1, 1e-4, "f32", bit_depth=12, handle=hd)
        n = 200 if w * h <= 4 << 20 else 50
        t_norm = _timed(lambda: ofv.stage_normalize(frame, 1, 1e-4, "f32", bit_depth=12, handle=hd), n, 5)
        t_pyr = _timed(lambda: ofv.stage_pyramid(plane, 3, handle=hd), n, 5)
        px = w * h
        norm_bytes = px * (2 + 4)
        pyr_bytes = px * 4 + sum(((w + (1 << k) - 1) >> k) * ((h + (1 << k) - 1) >> k) * 4 for k in (1, 2, 3))
        rows.append({"size": f"{w}x{h}", "normalize_us": round(t_norm * 1e6, 2),
                     "normalize_GBps": round(norm_bytes / t_norm / 1e9, 1),
                     "pyramid3_us": round(t_pyr * 1e6, 2), "pyramid3_GBps": round(pyr_bytes / t_pyr / 1e9, 1)})
        hd.close()
    return {"metric": "normalisation and three-level pyramid of one frame (host-timed, per call)", "rows": rows,
            "data": "uniform random 12-bit frames"}


def run_suite(args):
    import torch
    import paper_2509_25924_amd as ofv
    from paper_2509_25924_amd import _build
    if not _build.built():
        _build.build()
    ofv.load()
    dev = torch.device("cuda:0")
    names = (["batch4mp", "live21mp", "stream21mp", "sweep", "estimators", "adjoint512", "paper"] if args.suite == "all"
             else [args.suite])
    fns = {"batch4mp": suite_batch4mp, "live21mp": suite_live21mp, "stream21mp": suite_stream21mp,
           "sweep": suite_sweep, "estimators": suite_estimators, "oracle": suite_oracle,
           "adjoint512": suite_adjoint512, "paper": suite_paper, "preprocess": suite_preprocess,
           "livestep": suite_livestep}
    for nm in names:
        print(f"# suite {nm} ...", file=sys.stderr, flush=True)
        r = fns[nm](args, dev)
        r["suite"] = nm
        print(json.dumps(r), flush=True)


def time_two_streams(make_step, handles, steps, warmup):
    """Consecutive steps alternate between two handles, each with its own stream and its own captured
    graph(s), so that one step's normalisation, pyramid and coarse levels overlap the other's
    Gauss-Newton launches (no dependency joins the two streams; each handle owns its workspace).
    make_step(handle, i) returns a list of graph-capturable callables (one per input set); step k
    replays set k // 2 of handle k % 2.  Returns seconds per step."""
    import torch
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    graphs = []
    for i, hd in enumerate(handles):
        s = streams[i]
        fns = make_step(hd, i)
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for fn in fns:
                fn()
        gs = []
        for fn in fns:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                fn()
            gs.append(g)
        graphs.append(gs)
    torch.cuda.synchronize()
    k = [0]

    def step():
        i = k[0] % 2
        gs = graphs[i]
        with torch.cuda.stream(streams[i]):
            gs[(k[0] // 2) % len(gs)].replay()
        k[0] += 1
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    del graphs
    return sec


def time_gn_launch(ofv, p0, p1, fin, kr, reg_rel, reg_abs, handle, n, graph=True):
    """Average duration of one full-resolution Gauss-Newton launch (the stage entry point, same launch
    configuration and decomposition as inside the pipeline): n launches captured back to back in a hipGraph,
    each reading the field the previous one wrote and writing the other of two buffers, as the pipeline's
    iterations do; each of five replays bracketed by HIP events on the stream the kernel is launched on,
    median replay.  Also returns an eager loop of the same calls and event pairs around single eager
    launches."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    bufs = [fin.clone(), torch.empty_like(fin)]

    def launch(i):
        ofv.stage_gn_iteration(p0, p1, bufs[i % 2], "direct", kr, reg_rel, reg_abs, handle=handle,
                               out=bufs[(i + 1) % 2])

    def reset():
        bufs[0].copy_(fin)
    for i in range(3):
        launch(i)
    reset()
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(evs):
        a.record()
        launch(i)
        b.record()
    torch.cuda.synchronize()
    pair_s = sum(a.elapsed_time(b) for a, b in evs) / 1e3 / n
    reset()
    ev0.record()
    for i in range(n):
        launch(i)
    ev1.record()
    torch.cuda.synchronize()
    eager_s = ev0.elapsed_time(ev1) / 1e3 / n
    kern_s = eager_s
    if graph:
        reset()
        kgraph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(kgraph):
            for i in range(n):
                launch(i)
        handle.bind_stream()
        kgraph.replay()
        torch.cuda.synchronize()
        reps = []
        for _ in range(5):
            ev0.record()
            kgraph.replay()
            ev1.record()
            torch.cuda.synchronize()
            reps.append(ev0.elapsed_time(ev1))
        kern_s = sorted(reps)[len(reps) // 2] / 1e3 / n
        del kgraph
    return kern_s, eager_s, pair_s


def tuned_decomposition(handle, kr, w, h):
    """Name of the tuned decomposition of the level-0 direct-flow launch, 'auto' if none; a band entry with a
    fixed tile height carries it ('band/h128'), one sized from the occupancy at launch is plain 'band'."""
    for line in handle.tuning_table().splitlines():
        f = [int(x) for x in line.split()]
        if f[0] == kr and f[2] == 1 and f[3] == w and f[4] == h and f[5] == 1:
            return GN_NAMES[f[6]] + (f"/h{f[7]}" if f[6] == 11 and f[7] > 0 else "")
    return "auto"


def valu_ceiling(workload, storage, decomp, px, kern_s):
    """VALU issue ceiling of the launch: its instructions per pixel (committed SQ_INSTS_VALU summary for the
    current kernel sources) at the chip's non-packed issue rate, and the fraction of that ceiling reached."""
    instr = measured_traffic(workload, storage, decomp, kind="valu")
    if instr is None:
        return None
    per_px = instr * 64 / px               # wavefront instructions x 64 lanes
    ceil_s = px * per_px / VALU_LANE_INSTR_PER_S
    return {"bound": "alu", "instr_per_px": round(per_px, 1), "peak": VALU_LANE_INSTR_PER_S,
            "unit": "lane-instr/s", "ceiling_us": round(ceil_s * 1e6, 3), "frac": round(ceil_s / kern_s, 4),
            "note": "time the launch would take issuing its VALU instructions at the non-packed issue rate, "
                    "over its measured duration"}


def wake_21mp_setup(dev, storage, autotune=True):
    """5120x4096 12-bit cylinder-wake pair (the live workload's frame) on the device, its normalised planes,
    a handle tuned on the pair, and the estimated field as the input flow of the level-0 launch."""
    import paper_2509_25924_amd as ofv
    import synth
    from synth.gpu_render import make_pair_device
    W, H = 5120, 4096
    flow = synth.CylinderWake(H, W, t=0.0, dmax=10.0)
    a, b, _ = make_pair_device(H, W, flow, fwhm=2.5, ppp=0.1, seed=4000, bit_depth=12, noise=0.01 * 4095,
                               device=dev, max_disp=10.0, with_gt=False)
    prm = {"num_levels": 4, "kernel_radius": 10, "iterations": 3, "norm_radius": 2, "storage": storage}
    hd = ofv.Handle(W, H, 1)
    if autotune:
        fin = hd.autotune(a, b, prm, bit_depth=12, repeats=3)
    else:
        fin = ofv.compute_flow(a, b, prm, bit_depth=12, handle=hd)
    p0 = ofv.stage_normalize(a, 2, 1e-4, storage, bit_depth=12, handle=hd)
    p1 = ofv.stage_normalize(b, 2, 1e-4, storage, bit_depth=12, handle=hd)
    return hd, p0, p1, fin.contiguous(), prm


def roofline_21mp(dev, storage, launches):
    """Roofline of the level-0 Gauss-Newton launch at 5120x4096 (KR 10): about 500 MB per launch (FP32), far
    above the 256 MB Infinity Cache, so the bytes stream from HBM."""
    import torch
    W, H = 5120, 4096
    hd, p0, p1, fin, prm = wake_21mp_setup(dev, storage)
    decomp = tuned_decomposition(hd, 10, W, H)
    kern_s, eager_s, _ = time_gn_launch(__import__("paper_2509_25924_amd"), p0, p1, fin, 10, 1e-3, 1e-9, hd,
                                        launches)
    s_bytes = 4 if storage == "f32" else 2
    byts = (2 * s_bytes + 16) * W * H
    achieved = byts / kern_s / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": measured_traffic("wake_21mp", storage, decomp),
           "kernel": f"Gauss-Newton iteration, {decomp}, KR 10, {storage}, full resolution {W}x{H}",
           "bytes_per_launch": byts, "us_per_launch": round(kern_s * 1e6, 3), "launches_timed": launches,
           "timed_as": "median of 5 hipGraph replays of back-to-back launches",
           "us_eager_loop_per_launch": round(eager_s * 1e6, 3),
           "workload": "5120x4096 12-bit cylinder-wake pair (live workload frame), L 4, KR 10, IT 3, NR 2; "
                       "input flow = the estimated field"}
    out["valu"] = valu_ceiling("wake_21mp", storage, decomp, W * H, kern_s)
    hd.close()
    del p0, p1, fin
    torch.cuda.empty_cache()
    return out


def pmc_probe_21mp(args, dev):
    """For hardware-counter runs: the 256 MiB elementwise negation and copy (calibration), then the
    5120x4096 level-0 Gauss-Newton launch (KR 10) 5 times in every decomposition that fits KR 10."""
    import torch
    import paper_2509_25924_amd as ofv
    hd, p0, p1, fin, prm = wake_21mp_setup(dev, args.storage, autotune=False)
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    bufs = [fin.clone(), torch.empty_like(fin)]     # the field ping-pongs between two buffers, as in the pipeline
    for variant in GN_NAMES.values():
        hd.set_gn_variant(variant)
        bufs[0].copy_(fin)
        for i in range(5):
            ofv.stage_gn_iteration(p0, p1, bufs[i % 2], "direct", 10, 1e-3, 1e-9, handle=hd, out=bufs[(i + 1) % 2])
        torch.cuda.synchronize()
    s_bytes = 4 if args.storage == "f32" else 2
    print(json.dumps({"pmc_probe": "wake_21mp", "copy_bytes_each_way": src.numel() * 4,
                      "gn_bytes_per_launch": (2 * s_bytes + 16) * 5120 * 4096}))


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this estimator build has no multi-GPU path "
              "(independent pairs shard across GPUs with no communication); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.suite:
        run_suite(args)
        return

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
    if args.workload == "wake_21mp":
        if not args.pmc_probe:
            print("--workload wake_21mp is for --pmc-probe runs (the headline's 21 Mp roofline measures it "
                  "otherwise)", file=sys.stderr)
            sys.exit(2)
        pmc_probe_21mp(args, dev)
        return
    pair, prm, desc, bits = workload(args.workload)
    prm = dict(prm, storage=args.storage)
    h, w = pair.frame0.shape
    f0 = torch.from_numpy(pair.frame0).to(dev)
    f1 = torch.from_numpy(pair.frame1).to(dev)
    out = torch.empty((2, h, w), dtype=torch.float32, device=dev)
    handle = ofv.Handle(w, h, 1)
    if args.variant == "tuned":
        if args.tuning_table:
            with open(args.tuning_table) as fh:
                handle.load_tuning_table(fh.read())
        elif not args.pmc_probe:
            handle.autotune(f0, f1, prm, bit_depth=bits, repeats=7)
        if args.save_tuning:
            with open(args.save_tuning, "w") as fh:
                fh.write(handle.tuning_table())
    else:
        handle.set_gn_variant(args.variant)

    def step():
        ofv.compute_flow(f0, f1, prm, bit_depth=bits, out=out, handle=handle)

    if args.pmc_probe:
        step()
        p0 = ofv.stage_normalize(f0, prm["norm_radius"], prm["norm_eps"], args.storage, bit_depth=bits, handle=handle)
        p1 = ofv.stage_normalize(f1, prm["norm_radius"], prm["norm_eps"], args.storage, bit_depth=bits,
                                 handle=handle)
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.neg(src, out=dst)     # elementwise kernel: 256 MiB read, 256 MiB written
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)              # runtime blit kernel, same bytes
        torch.cuda.synchronize()
        fin = out.clone()
        bufs = [fin.clone(), torch.empty_like(fin)]  # the field ping-pongs between two buffers, as in the pipeline
        for variant in GN_NAMES.values():
            handle.set_gn_variant(variant)
            bufs[0].copy_(fin)
            for i in range(5):
                ofv.stage_gn_iteration(p0, p1, bufs[i % 2], "direct", prm["kernel_radius"], prm["reg_rel"],
                                       prm["reg_abs"], handle=handle, out=bufs[(i + 1) % 2])
            torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": args.workload, "copy_bytes_each_way": src.numel() * 4,
                          "gn_bytes_per_launch": (2 * (4 if args.storage == "f32" else 2) + 16) * w * h}))
        return

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

    # ---- two streams: pairs alternate between two handles, so that one pair's
    # normalisation, pyramid and small coarse-level launches overlap the other's
    # Gauss-Newton launches (context beside the serial figure above)
    two_stream = None
    if graph is not None:
        h2 = ofv.Handle(w, h, 1)
        if args.variant == "tuned":
            h2.load_tuning_table(handle.tuning_table())
        else:
            h2.set_gn_variant(args.variant)
        outs2 = [out, torch.empty_like(out)]

        def make_step(hd, i):
            return [lambda: ofv.compute_flow(f0, f1, prm, bit_depth=bits, out=outs2[i], handle=hd)]
        sec2 = time_two_streams(make_step, [handle, h2], args.steps, args.warmup)
        for o in outs2:
            if not torch.equal(o, eager_ref):
                raise RuntimeError("two-stream replay differs from the eager result")
        two_stream = {"fields_per_s": round(1.0 / sec2, 1), "mvectors_per_s": round(w * h / sec2 / 1e6, 1),
                      "ms_per_pair": round(sec2 * 1e3, 5), "speedup_over_serial": round(sec / sec2, 3),
                      "how": "pairs alternate between two handles on two streams (hipGraph each); the serial "
                             "figure is the headline value"}
        handle.bind_stream()

    # ---- dominant kernel: Gauss-Newton iteration at full resolution, same
    # launch configuration as inside the pipeline, timed with HIP events on
    # the stream it is launched on (torch's current stream, bound to the handle).
    kr = prm["kernel_radius"]
    p0 = ofv.stage_normalize(f0, prm["norm_radius"], prm["norm_eps"], args.storage, bit_depth=bits, handle=handle)
    p1 = ofv.stage_normalize(f1, prm["norm_radius"], prm["norm_eps"], args.storage, bit_depth=bits, handle=handle)
    fin = out.clone()
    kern_s, eager_s, pair_s = time_gn_launch(ofv, p0, p1, fin, kr, prm["reg_rel"], prm["reg_abs"], handle,
                                             args.kernel_launches, graph=graph is not None)
    # practical HBM ceiling for context: a 256 MiB device-to-device copy (512 MiB moved), event-timed
    csrc = torch.empty(64 << 20, dtype=torch.float32, device=dev)
    cdst = torch.empty_like(csrc)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        cdst.copy_(csrc)
    ev0.record()
    for _ in range(10):
        cdst.copy_(csrc)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbps = 10 * 2 * csrc.numel() * 4 / (ev0.elapsed_time(ev1) / 1e3) / 1e9
    del csrc, cdst
    decomp = args.variant
    if args.variant == "tuned":
        decomp = tuned_decomposition(handle, kr, w, h)
    if decomp == "auto":
        decomp = "march" if w * h >= (3 << 20) else "tile64x16"
    s_bytes = 4 if args.storage == "f32" else 2
    bytes_per_px = 2 * s_bytes + 16            # P0, P1, V in, V out
    algo_bytes = bytes_per_px * w * h
    achieved = algo_bytes / kern_s / 1e9

    # whole-step algorithmic bytes for context: the per-sweep model and the fused-iteration lower bound
    L, it = prm["num_levels"], prm["iterations"]
    in_bytes = {8: 1, 12: 2, 16: 2}.get(bits, 4)
    step_bytes = _sweep_bytes(L, w, h, it, s_bytes, in_bytes)
    step_fused = _sweep_bytes(L, w, h, 1, s_bytes, in_bytes)

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
        "two_stream_pipeline": two_stream,
        "step_algorithmic_GBps": round(step_bytes / sec / 1e9, 1),
        "step_bytes_models": _step_models(step_bytes, step_fused, sec),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.workload, args.storage, decomp),
                     "kernel": f"Gauss-Newton iteration, {decomp}, KR {kr}, {args.storage}, full resolution {w}x{h}",
                     "bytes_per_launch": algo_bytes, "us_per_launch": round(kern_s * 1e6, 3),
                     "launches_timed": args.kernel_launches,
                     "timed_as": "median of 5 hipGraph replays of back-to-back launches" if graph is not None else "eager loop",
                     "us_eager_loop_per_launch": round(eager_s * 1e6, 3),
                     "us_event_pair_per_launch": round(pair_s * 1e6, 3),
                     "stream_copy_GBps": round(copy_gbps, 1),
                     "working_set_MB": round(algo_bytes / 1e6, 1),
                     "cache_resident": "the launch's working set fits the 256 MB Infinity Cache, so back-to-back "
                                       "launches are served partly from it; roofline_21mp is the HBM-bound "
                                       "measurement",
                     "valu": valu_ceiling(args.workload, args.storage, decomp, w * h, kern_s)},
    }
    if not args.no_21mp:
        for st in ("f32", "bf16"):
            result[f"roofline_21mp_{st}"] = roofline_21mp(dev, st, 20)

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
                                            f"({t_cpu:.1f} s)", "host": host_cpu()}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
