"""Benchmark of the RAPID refinement sweep on one MI355X.

A step is one whole segmentation (block-sum pyramid, grid, every level,
stage and sweep of the refinement, and the gate's features and network when
gated; pixel labels written) with the input already resident in HBM.  The
default workload is the whole-slide one: a 65536 x 49152 synthetic H&E slide
(3.22 GPixel, 40 % background) cut into 768 tiles of 2048^2 with a 64-px
halo, 32-px superpixel cells (3,145,728 superpixels), three levels of ratio
4 (effective blocks 16 | 8, 4 | 2, 1), all tiles in one launch; plain, then
under the learned prediction gate at the thresholds calibrated on held-out
tiles for boundary recall >= 0.99 and >= 0.995 against the plain labels.

Prints one JSON line: plain throughput in MPixel/s (value), the gated
points, the roofline of the refinement kernel (HBM-bound: there is no dense
contraction on the sweep), and the CPU oracle timed on sampled tiles of the
same slide on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MPixel/s segmented (all levels) at 1 MI355X, gated vs plain, % HBM peak"


def kernel_source_hash() -> str:
    """Hash of the device code the profiles were taken on: the kernel
    sources with comments, trailing blanks and empty lines removed, so that
    a change of wording leaves the figures valid and a change of code does
    not."""
    h = hashlib.sha256()
    for f in ("rapid_kernels.hip", "rapid_internal.h", "rapid_gate_dev.h"):
        with open(os.path.join(ROOT, "paper_1704_02083_amd", "csrc", f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        lines = [l.rstrip() for l in src.split("\n")]
        h.update("\n".join(l for l in lines if l).encode())
    return h.hexdigest()[:16]


def workload(name: str):
    from paper_1704_02083_amd import params, synth
    if name == "slide":
        return None, params.default_params(2048, 2048, 4096, levels=params.THREE_LEVEL), (
            "whole-slide-like: 32768x32768 RGB uint8 synthetic H&E (40% background), 2048x2048 tiles "
            "with 64-px halo in one launch, 32-px cells (1,048,576 superpixels), three levels 16|8,4|2,1")
    if name == "slide65k":
        return None, params.default_params(2048, 2048, 4096, levels=params.THREE_LEVEL), (
            "whole-slide-like: 65536x49152 RGB uint8 synthetic H&E (3.22 GPixel, 40% background), 768 "
            "2048x2048 tiles with 64-px halo in one launch, 32-px cells (3,145,728 superpixels), three "
            "levels 16|8,4|2,1")
    if name == "he4096":
        return None, params.config3(gate_level=1), (
            "one 4096x4096 RGB uint8 synthetic H&E tile (30% background), K=16384, three levels 16|8,4|2,1")
    if name == "he8192":
        return None, params.config3(8192, 8192, 65536), (
            "one 8192x8192 RGB uint8 synthetic H&E image (30% background), K=65536, three levels 16|8,4|2,1")
    if name == "batch":
        imgs = synth.batch_images(200)
        p = params.config2(481, 321)
        desc = ("batched plain: 200 RGB uint8 images (100 481x321 + 100 321x481), Voronoi "
                "gradient mosaics, K=400, one level, blocks 16,8,4,2,1")
    elif name == "single256":
        imgs = [synth.voronoi_blur()]
        p = params.config1()
        desc = "plain: one 256x256 RGB uint8 Voronoi image, K=64, blocks 16,8,4,2,1, min 64 px"
    else:
        raise SystemExit("unknown workload " + name)
    return imgs, p, desc


PYRAMID_MIN_JOBS = 128   # from this many images or tiles the refinement kernel builds the pyramids


def stage_bytes(W, H, rep, pyramid: bool) -> int:
    """Algorithmic bytes of the stages of one image or tile: the traffic the
    method cannot avoid, from its per-stage counters.  With the block-sum
    pyramid built inside the launch, the RGB pixels are read once (3 B per
    pixel).  Each stage scans its label map once for the boundary blocks
    (4 B per block; a gated stage with nothing to do reads nothing); each
    block visit reads the block's colour sum (6 B: three 16-bit channels);
    each commit writes a label (4 B) and moves the size, colour and position
    sums of two superpixels (96 B: 2 x 6 words of 8 B)."""
    total = 3 * W * H if pyramid else 0
    for r in rep:
        B = r["block"]
        nb = -(-W // B) * -(-H // B)
        if r["active"] or r["sweeps"]:
            total += 4 * nb
        total += 6 * r["active"] + (4 + 96) * r["commits"]
    return total


def stage_bytes_window(W, H, rep, pyramid: bool) -> int:
    """A second, larger byte model of the same stages, closer to what the
    kernel reads: with the pyramid, 3 B per pixel read plus 8 B per block of
    every stage with B >= 2 written; per stage 8 B per block (the label map
    written once and scanned once); per block visit its whole 3x3 label
    window (36 B) and its packed colour sum (8 B; 3 B at B = 1); per commit a
    label (4 B) and the sum again; statistics on chip (0 B)."""
    total = 3 * W * H if pyramid else 0
    for r in rep:
        B = r["block"]
        nb = -(-W // B) * -(-H // B)
        sb = 3 if B == 1 else 8
        total += 8 * nb + r["active"] * (36 + sb) + r["commits"] * (4 + sb)
        if B >= 2 and pyramid:
            total += 8 * nb
    return total


def refine_alg_bytes(imgs, reports, model=stage_bytes, pyramid: bool | None = None) -> float:
    """Algorithmic bytes of one refinement launch over whole images: the
    stages' bytes plus the final pixel labels written once (4 B per pixel).
    pyramid: whether the launch builds the block-sum pyramid itself (its
    reported launch shape); None: as a batch launch decides it."""
    if pyramid is None:
        pyramid = len(imgs) >= PYRAMID_MIN_JOBS
    total = 0
    for img, rep in zip(imgs, reports):
        H, W = img.shape[:2]
        total += 4 * W * H + model(W, H, rep, pyramid)
    return float(total)


def tiles_alg_bytes(W, H, tiles, reports, model=stage_bytes) -> float:
    """As refine_alg_bytes for the tiles of a slide: the stages run over each
    tile's extended rectangle (core plus halo), the final labels are written
    for the core pixels only, so once per slide pixel."""
    total = 4 * W * H
    for t, rep in zip(tiles, reports):
        x0, y0, x1, y1 = t["ext"]
        total += model(x1 - x0, y1 - y0, rep, len(tiles) >= PYRAMID_MIN_JOBS)
    return float(total)


def host_cpu() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def device_facts() -> dict:
    """The GPU the line was measured on, as the runtime reports it."""
    import torch
    pr = torch.cuda.get_device_properties(0)
    out = {"name": pr.name, "arch": getattr(pr, "gcnArchName", ""), "compute_units": pr.multi_processor_count,
           "memory_gib": round(pr.total_memory / 2 ** 30, 1)}
    l2 = getattr(pr, "L2_cache_size", None)
    if l2:
        out["l2_mib"] = round(l2 / 2 ** 20, 1)
    return out


def profile_traffic(kernel: str, wl: str, src_hash: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "%s_%s_counters.txt" % (kernel, wl))
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_hash:\s*(\w+)", txt)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != src_hash:
        return None
    return float(t.group(1))


def _oracle_worker(idx, p, barrier, results):
    """One process of the multi-core CPU baseline: generates the batched
    workload's images idx from their seeds, waits for the other processes,
    then times the oracle on them (wall clock, comparable across processes)."""
    import oracle
    from paper_1704_02083_amd import synth
    imgs = [synth.voronoi_gradient(*((481, 321) if i < 100 else (321, 481)), seed=1000 + i) for i in idx]
    barrier.wait(timeout=300)
    t0 = time.time()
    for img in imgs:
        oracle.segment(img, p)
    results.put((sum(im.shape[0] * im.shape[1] for im in imgs), t0, time.time()))


def cpu_baseline_multicore(p, n_images: int = 200):
    """The oracle in independent processes over the 200 batched images, one
    process per core the host grants (at most 16): a multi-core host
    throughput beside the single-threaded one.  The processes are fresh
    interpreters, so they hold no GPU state."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("spawn")
    barrier, results = ctx.Barrier(cores), ctx.Queue()
    procs = [ctx.Process(target=_oracle_worker, args=(list(range(c, n_images, cores)), p, barrier, results))
             for c in range(cores)]
    for pr in procs:
        pr.start()
    got = [results.get(timeout=600) for _ in procs]
    for pr in procs:
        pr.join()
    px = sum(g[0] for g in got)
    dt = max(g[2] for g in got) - min(g[1] for g in got)
    return {"value": round(px / dt / 1e6, 4), "unit": "MPixel/s", "cores": cores, "kind": "oracle",
            "sample": "all %d images, %d independent processes, %.1f s" % (n_images, cores, dt)}


def cpu_baseline(imgs, p, sample: int):
    import oracle
    oracle.build()
    n = min(sample, len(imgs))
    px = 0
    t0 = time.perf_counter()
    for img in imgs[:n]:
        oracle.segment(img, p)
        px += img.shape[0] * img.shape[1]
    dt = time.perf_counter() - t0
    out = {"value": round(px / dt / 1e6, 4), "unit": "MPixel/s", "cores": 1, "kind": "oracle",
           "sample": "%d of the %d images (%d px), single-threaded, %.1f s" % (n, len(imgs), px, dt),
           "host_cpu": host_cpu()}
    if not p.get("merge"):
        # the oracle's sequential FIFO-queue schedule (the paper's queue read
        # literally) on the same sample: context for the synchronous one
        t0 = time.perf_counter()
        for img in imgs[:n]:
            oracle.segment_fifo(img, p)
        out["fifo_schedule_value"] = round(px / (time.perf_counter() - t0) / 1e6, 4)
    return out


def _oracle_tile_worker(sub, p, barrier, results):
    """One process of the multi-core CPU baseline on slide tiles: waits for
    the other processes, then times the oracle on its tile (wall clock)."""
    import oracle
    barrier.wait(timeout=300)
    t0 = time.time()
    oracle.segment(sub, p)
    results.put((t0, time.time()))


def cpu_baseline_tiles(rgb, W, H, p, lay, n_single: int = 8):
    """The oracle on sampled tiles of the slide, each an independent image
    over its core plus halo as in the launch: single-threaded over n_single
    tiles spread over the slide (the first and last tile, the rest evenly
    between them), as a slide rate of core pixels per second (the slide
    takes 768 / n_single times their time); and one distinct tile per core
    the host grants (at most 16) in independent processes, as a multi-core
    host rate.  Generation and copies are outside the timed regions."""
    import multiprocessing as mp
    import numpy as np
    import oracle
    oracle.build()

    def tile_case(i):
        t = lay[i]
        ex0, ey0, ex1, ey1 = t["ext"]
        cx0, cy0, cx1, cy1 = t["core"]
        sub = np.ascontiguousarray(rgb[ey0:ey1, ex0:ex1].cpu().numpy())
        return sub, dict(p, K=0, gx=t["gx"], gy=t["gy"]), (cx1 - cx0) * (cy1 - cy0)

    idx = sorted({int(round(x)) for x in np.linspace(0, len(lay) - 1, n_single)})
    cases = [tile_case(i) for i in idx]
    t0 = time.perf_counter()
    for sub, pt, _ in cases:
        oracle.segment(sub, pt)
    dt = time.perf_counter() - t0
    core = sum(c[2] for c in cases)
    ext = sum(c[0].shape[0] * c[0].shape[1] for c in cases)
    out = {"value": round(core / dt / 1e6, 4), "unit": "MPixel/s", "cores": 1, "kind": "oracle",
           "sample": "%d of the %d tiles (indices %s; %.1f MPixel of core, %.1f with halos), single-threaded, "
                     "%.1f s; the whole slide would take %.0f s at this rate"
                     % (len(idx), len(lay), idx, core / 1e6, ext / 1e6, dt, dt * W * H / core),
           "host_cpu": host_cpu()}
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    midx = sorted({int(round(x)) for x in np.linspace(1, len(lay) - 2, cores)})
    mcases = [tile_case(i) for i in midx]
    ctx = mp.get_context("spawn")
    barrier, results = ctx.Barrier(len(mcases)), ctx.Queue()
    procs = [ctx.Process(target=_oracle_tile_worker, args=(sub, pt, barrier, results)) for sub, pt, _ in mcases]
    for pr in procs:
        pr.start()
    got = [results.get(timeout=900) for _ in procs]
    for pr in procs:
        pr.join()
    wall = max(g[1] for g in got) - min(g[0] for g in got)
    mcore = sum(c[2] for c in mcases)
    out["multicore"] = {"value": round(mcore / wall / 1e6, 4), "unit": "MPixel/s", "cores": len(mcases),
                        "kind": "oracle",
                        "sample": "%d distinct tiles (%.1f MPixel of core), one per process, %.1f s"
                                  % (len(mcases), mcore / 1e6, wall)}
    return out


def timed_steps(ctx, step, args):
    """W untimed warm-up steps (plus one untimed call that tunes the launch
    shape when the autotuner is on and W = 0), then K steps back to back
    (launches queue while the GPU works) between two synchronisations.
    Returns the wall time per step, the refinement kernel's duration in each
    of the K timed steps (HIP events the library records on its stream, read
    after the timed region), and whether a tuning call was added."""
    import torch
    tune_call = args.warmup == 0 and not args.no_autotune
    for _ in range(args.warmup + (1 if tune_call else 0)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    return dt, ctx.timing_history(args.steps), tune_call


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="slide65k", choices=["batch", "single256", "he4096", "he8192", "slide",
                                                                "slide65k", "roi"])
    ap.add_argument("--gated", action="store_true",
                    help="he4096 and slide: also train the gate and time the gated path (slide65k: always)")
    ap.add_argument("--no-gated", action="store_true", help="slide65k: the plain path only")
    ap.add_argument("--gate-rule", default="both", choices=["either", "both"])
    ap.add_argument("--save-gate", default=None, help="write the trained gate network to this .npz file")
    ap.add_argument("--gate-level", type=int, default=3, choices=[1, 2, 3],
                    help="level of the schedule 16 | 8,4 | 2 | 1 from which the gate applies")
    ap.add_argument("--train-tiles", type=int, default=64, help="4096x4096 training tiles of the gate")
    ap.add_argument("--min-miss", type=int, default=1,
                    help="gate target: a superpixel is positive from this many boundary pixels that "
                         "freezing it at the gate point would miss")
    ap.add_argument("--grain", type=int, default=1,
                    help="H&E workloads: stop the schedule at this effective block size (the paper's "
                         "'grain'; 4 = its 4x4 setting)")
    ap.add_argument("--merge", action="store_true",
                    help="batch and single256: merge on underflow (Sec. 3.1, Eqs. (4)-(5)); the "
                         "line also reports the merges and the boundary recall against the plain labels")
    ap.add_argument("--reuse-baseline", action="store_true",
                    help="he4096: also time the level-by-level path with the statistics carried "
                         "across levels (Sec. 3.2) against recounting them from the pixels at "
                         "every level (multi-scale CTFTPS without reuse)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default launch shape instead of the autotuned one (the first "
                         "warm-up step tunes)")
    ap.add_argument("--cpu-sample", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy three times (scales the HBM "
                         "byte counters of rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.steps < 1 or args.warmup < 0:
        raise SystemExit("--steps must be >= 1 and --warmup >= 0")
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the refinement path runs on a single MI355X "
              "(the library shards no work across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1704_02083_amd import rapid

    if args.copy_calibration:
        # a plain 1 GiB device copy: scales the byte counters of rocprofv3
        # --pmc, and its rate is the achievable HBM bandwidth to set beside
        # the 8 TB/s peak (read + write bytes over the copy's duration)
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        print(json.dumps({"copy_calibration_bytes": n, "launches": 4, "copy_ms": round(ms, 4),
                          "copy_GBps": round(2 * n / (ms * 1e-3) / 1e9, 1)}), flush=True)
        return

    if args.workload in ("slide", "slide65k", "he4096", "he8192"):
        return bench_he(args)
    if args.workload == "roi":
        return bench_roi(args)

    imgs, p, desc = workload(args.workload)
    if args.merge:
        p = dict(p, merge=True)
        desc += ", merge on underflow"
    print("bench: workload %s, %d images generated" % (args.workload, len(imgs)), file=sys.stderr,
          flush=True)
    rgbs = [torch.from_numpy(im).cuda() for im in imgs]
    labels = [torch.empty(im.shape[:2], dtype=torch.int32, device="cuda") for im in imgs]
    ctx = rapid.Context(0, timing=True, autotune=not args.no_autotune)
    pixels = sum(im.shape[0] * im.shape[1] for im in imgs)

    def step():
        if len(rgbs) == 1:
            ctx.segment(rgbs[0], p, labels=labels[0], report=False)
        else:
            ctx.segment_batch(rgbs, p, labels=labels, report=False)

    dt, refine_ms, tune_call = timed_steps(ctx, step, args)
    dt *= args.steps
    print("bench: timed %d steps in %.3f s" % (args.steps, dt), file=sys.stderr, flush=True)
    tm = ctx.last_timings()
    shape = {"threads": tm["threads"], "stats_lds": tm["stats_lds"], "pyramid_in_launch": tm["pyramid"],
             "workgroups_per_image": tm["workgroups"], "autotuned": not args.no_autotune}
    # one image spread over a cooperative launch runs the k_refine_mc kernel
    kname = "k_refine_mc" if tm["workgroups"] > 1 else "k_refine"

    # counters of the same (deterministic) work, from one untimed call
    if len(rgbs) == 1:
        _, r = ctx.segment(rgbs[0], p, labels=labels[0], report=True)
        reps = [r]
    else:
        _, reps = ctx.segment_batch(rgbs, p, labels=labels, report=True)
    ms_step = dt * 1e3 / args.steps
    avg_refine = sum(refine_ms) / len(refine_ms)
    alg = refine_alg_bytes(imgs, reps, pyramid=bool(tm["pyramid"]))
    alg_w = refine_alg_bytes(imgs, reps, stage_bytes_window, pyramid=bool(tm["pyramid"]))
    achieved = alg / (avg_refine * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    traffic = profile_traffic(kname, args.workload + ("_merge" if args.merge else ""), src_hash)
    out = {
        "metric": METRIC,
        "value": round(pixels * args.steps / dt / 1e6, 3),
        "unit": "MPixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": desc, "images": len(imgs), "pixels": pixels,
                   "superpixels_per_image": p["K"], "path": "plain+merge" if args.merge else "plain"},
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": round(achieved, 3),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 6),
            "traffic": traffic,
            "alg_bytes_per_launch": alg,
            "avg_launch_ms": round(avg_refine, 4),
            "launches_timed": len(refine_ms),
            "window_model": {"alg_bytes_per_launch": alg_w,
                             "frac": round(alg_w / (avg_refine * 1e-3) / 1e9 / HBM_PEAK_GBS, 6)},
            "source_hash": src_hash,
        },
        "launch_shape": shape,
        "autotune_call": tune_call,
    }
    if args.merge:
        # what the merges did: superpixels merged away, and how many of the
        # plain segmentation's boundary pixels the merged one still has
        # within 2 px (boundary recall, Sec. 4.2)
        merges = sum(r["merges"] for rep in reps for r in rep)
        plain = [torch.empty_like(l) for l in labels]
        if len(rgbs) == 1:
            ctx.segment(rgbs[0], dict(p, merge=False), labels=plain[0], report=False)
        else:
            ctx.segment_batch(rgbs, dict(p, merge=False), labels=plain, report=False)
        nb = nm = 0
        for a, b in zip(plain, labels):
            _, x, y = ctx.boundary_miss(a, b, radius=2, counts=False)
            nb += x
            nm += y
        out["merge"] = {"merges": int(merges), "merges_per_image": round(merges / len(imgs), 2),
                        "boundary_recall_vs_plain": round(1.0 - nm / max(nb, 1), 5)}
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(imgs, p, args.cpu_sample)
        if args.workload == "batch":
            print("bench: timing the CPU oracle on all host cores", file=sys.stderr, flush=True)
            out["cpu_baseline"]["multicore"] = cpu_baseline_multicore(p)
    ctx.close()
    out["device"] = device_facts()
    print(json.dumps(out), flush=True)


def train_gate(ctx, rule: str, n_tiles: int, seed: int = 0, gate_level: int = 3, save: str | None = None,
               min_miss: int = 1):
    """Gate network trained on n_tiles synthetic 4096x4096 H&E tiles (seeds
    5000...) with 32-px cells: features and targets (a superpixel is
    positive from min_miss missed boundary pixels) from plain runs, the
    training itself, all on the GPU through the C-ABI."""
    import torch
    from paper_1704_02083_amd import gate, params, synth_gpu
    p = params.gated(4096, 4096, 16384, rule=rule, gate_level=gate_level)
    Xs, ts = [], []
    for i in range(n_tiles):
        rgb = synth_gpu.he_slide(4096, 4096, seed=5000 + i, background=0.4, device="cuda")
        X, t, _ = gate.tile_samples(ctx, rgb, p, min_miss=min_miss)
        Xs.append(X)
        ts.append(t)
        del rgb
    X, t = torch.cat(Xs), torch.cat(ts)
    t0 = time.perf_counter()
    master, w = gate.train(ctx, X, t, epochs=20, batch=4096, seed=seed)
    torch.cuda.synchronize()
    if save:
        gate.save_model(save, master, w, 0.0, gate_level, rule)
    return w, {"tiles": n_tiles, "samples": int(X.shape[0]), "min_miss": min_miss,
               "positive_rate": round(float(t.float().mean().item()), 4),
               "train_s": round(time.perf_counter() - t0, 3)}


def roofline(kname, alg, alg_w, launch_ms, traffic=None):
    """Roofline of the refinement kernel: algorithmic bytes per launch over
    its mean HIP-event duration against the HBM peak; the window model's
    figures beside it."""
    avg = sum(launch_ms) / len(launch_ms)
    achieved = alg / (avg * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic, "alg_bytes_per_launch": alg,
            "avg_launch_ms": round(avg, 4), "launches_timed": len(launch_ms),
            "window_model": {"alg_bytes_per_launch": alg_w,
                             "frac": round(alg_w / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 6)}}


def bench_gated(args, ctx, rgb, labels, plain, W, H, dt_plain):
    """The learned gate on the same image or slide: the gated schedule (the
    plain one with the single-pixel stage as its own, gated level), at the
    thresholds calibrated on held-out tiles for boundary recall >= 0.99 and
    >= 0.995 against the plain labels, beside the two references without a
    network decision: nothing refined past the gate point (the schedule
    stopped before the gated stage) and everything refined (the gate's
    overhead)."""
    import numpy as np
    import torch
    from paper_1704_02083_amd import gate, metrics, params, rapid, synth_gpu
    w, info = train_gate(ctx, args.gate_rule, args.train_tiles, gate_level=args.gate_level, save=args.save_gate,
                         min_miss=args.min_miss)
    print("bench: gate trained (%s)" % info, file=sys.stderr, flush=True)
    slide = args.workload in ("slide", "slide65k")
    if slide:
        pg = params.gated(2048, 2048, 4096, rule=args.gate_rule, gate_level=args.gate_level)
        lay = rapid.tile_layout(W, H, 2048, 64, 32)

        def run(th):
            ctx.segment_slide(rgb, pg, tile=2048, halo=64, cell=32, labels=labels, w_bf16=w, thresh=th)

        def report_run(th):
            _, reps, _, g = ctx.segment_slide(rgb, pg, tile=2048, halo=64, cell=32, labels=labels, w_bf16=w,
                                              thresh=th, report=True, features=True)
            return tiles_alg_bytes(W, H, lay, reps), tiles_alg_bytes(W, H, lay, reps, stage_bytes_window), g
    else:
        pg = params.gated(W, H, 16384, rule=args.gate_rule, gate_level=args.gate_level)

        def run(th):
            ctx.segment_gated([rgb], pg, w, th, labels=[labels], report=False)

        def report_run(th):
            _, reps, _, g = ctx.segment_gated([rgb], pg, w, th, labels=[labels], report=True)
            py = bool(ctx.last_timings()["pyramid"])
            return (refine_alg_bytes([rgb], reps, pyramid=py), refine_alg_bytes([rgb], reps, stage_bytes_window,
                                                                                 pyramid=py), g)
    hold = [synth_gpu.he_slide(2048, 2048, seed=7100 + i, background=0.4, device="cuda") for i in range(4)]
    crops = [(0, 0)] if not slide else [(1000, 3000), (9000, 17000), (20000, 7000), (28000, 28000)]
    measured = {}
    # the autotuner picks the gated launch's shape on its first call, for
    # every threshold after it: tune it on the heaviest case, everything
    # refined (untimed)
    run(-1e9)
    torch.cuda.synchronize()

    def point(th):
        if th in measured:
            return dict(measured[th])
        alg, alg_w, g = report_run(th)
        marked = float(g.to(torch.float32).mean().item())
        dt, ms, _ = timed_steps(ctx, lambda: run(th), args)
        ue = [metrics.undersegmentation_error(plain[y:y + 4096, x:x + 4096].cpu().numpy(),
                                              labels[y:y + 4096, x:x + 4096].cpu().numpy()) for y, x in crops]
        kname = "k_refine" if slide else "gated launches"
        tm = ctx.last_timings()
        r = {"thresh": th, "MPixel/s": round(W * H / dt / 1e6, 3), "ms_per_step": round(dt * 1e3, 3),
             "launch_shape": {"threads": tm["threads"], "stats_lds": tm["stats_lds"], "pyramid_in_launch": tm["pyramid"],
                              "workgroups_per_image": tm["workgroups"]},
             "speedup": round(dt_plain / dt, 4), "marked": round(marked, 6),
             "br": round(gate.boundary_recall(ctx, plain, labels), 6),
             "disagreement": round(float((plain != labels).float().mean().item()), 6),
             "ue": round(float(sum(ue) / len(ue)), 6),
             "roofline": roofline(kname, alg, alg_w, ms)}
        measured[th] = r
        print("bench: gated point thresh %g: %.1f MPixel/s, BR %.4f, marked %.4f"
              % (th, r["MPixel/s"], r["br"], marked), file=sys.stderr, flush=True)
        return dict(r)

    res = {"train": info, "rule": args.gate_rule,
           "schedule": "16 | 8,4 | 2 | 1, gate from level %d (%s)" % (
               args.gate_level, {3: "the 1-px stage", 2: "the 2-px and 1-px stages",
                                 1: "every stage after the 16-px one"}[args.gate_level]),
           "points": [], "references": []}
    for target in (0.99, 0.995):
        cal = gate.calibrate(ctx, hold, params.gated(2048, 2048, 4096, rule=args.gate_rule,
                                                     gate_level=args.gate_level), w, target,
                             candidates=[1e9, 4.0, 3.0, 2.0, 1.5, 1.25, 1.0, 0.75, 0.5, 0.4, 0.3, 0.2, 0.1, 0.0,
                                         -0.25, -0.5, -1.0, -2.0, -1e9])
        if cal is None:
            res["points"].append({"target_br": target, "calibrated": None})
            continue
        c = point(cal[0])
        c["target_br"] = target
        c["held_out"] = {k: round(v, 6) for k, v in cal[1].items()}
        # a threshold above every logit marks nothing: the target is then met
        # by stopping before the gated stage, with no decision of the network
        c["attribution"] = ("no network decision: nothing marked, the speedup is that of stopping before the "
                            "gated stage" if c["held_out"]["marked"] == 0.0 else
                            "network: the marked superpixels refine in the gated stage")
        res["points"].append(c)
    # what the network adds over a gate without it: on the held-out tiles, a
    # random choice of the same share of superpixels, and the share a random
    # choice needs to meet the target
    pg_h = params.gated(2048, 2048, 4096, rule=args.gate_rule, gate_level=args.gate_level)
    gx_h, gy_h = rapid.grid(2048, 2048, pg_h["K"])
    plain_h = [ctx.segment(r, pg_h, report=False)[0] for r in hold]

    def random_br(share):
        brs = []
        for i, (r, ph) in enumerate(zip(hold, plain_h)):
            K = gx_h * gy_h
            for sd in (0, 1):
                bits = np.zeros(K, np.uint8)
                bits[np.random.default_rng(1000 * sd + i).choice(K, int(round(share * K)), replace=False)] = 1
                lab_r, _ = ctx.segment(r, pg_h, gate=torch.from_numpy(bits).cuda(), report=False)
                brs.append(gate.boundary_recall(ctx, ph, lab_r))
        return float(np.mean(brs))

    for c in res["points"]:
        if c.get("calibrated", True) is None or c["held_out"]["marked"] == 0.0:
            continue
        m = c["held_out"]["marked"]
        need = None
        for share in [m] + [x for x in (0.6, 0.7, 0.8, 0.9, 1.0) if x > m]:
            br = random_br(share)
            if share == m:
                c["random_same_share"] = {"marked": round(m, 6), "br": round(br, 6)}
            if br >= c["target_br"]:
                need = share
                break
        c["random_share_for_target"] = need
        c["random_note"] = ("held-out tiles, two random gates per tile: boundary recall of a random choice of the "
                            "network's share, and the smallest share of (that share, 0.6 .. 1.0) whose random "
                            "choice meets the target")
    for name, th in (("nothing refined past the gate", 1e9), ("everything refined (gate overhead)", -1e9)):
        r = point(th)
        r["name"] = name
        res["references"].append(r)
    res["note"] = ("br and disagreement over the whole image against the plain labels, ue on %d 4096x4096 crops; "
                   "marked = share of superpixels whose gate bit is set; each point timed over the same warm-up "
                   "and step counts as the plain path" % len(crops))
    return res


def bench_roi(args):
    """The paper's own use of the prediction step: region-of-interest
    detection.  A classifier labels superpixels tissue or background at the
    second level, and past it only pairs across the predicted border refine
    (rule "differ").  Two classifiers, each the gate network trained on 16
    tiles (balanced batches): one on the paper's four ROI features (absolute
    and comparative brightness, extra- and intra-region dissimilarity,
    Sec. 4), one on the learned gate's sixteen.  Beside them the learned
    boundary-recall gate (rule "both", trained on where refinement moves
    boundaries) at the threshold whose boundary recall on the same tiles is
    the closest at or above the paper gate's.  16 held-out 2048x2048 H&E
    tiles in one launch, plain and gated; ROI masks (each pixel takes its
    superpixel's class from the four-feature classifier) scored against the
    generator's tissue mask."""
    import torch
    from paper_1704_02083_amd import gate, params, rapid, synth_gpu
    ctx = rapid.Context(0, timing=True)
    base = params.default_params(2048, 2048, 4096, levels=params.THREE_LEVEL, gate_level=1)
    train = [synth_gpu.he_slide(2048, 2048, seed=8000 + i, background=0.4, device="cuda") for i in range(16)]
    train_roi = [synth_gpu.tissue_mask(2048, 2048, seed=8000 + i, background=0.4) for i in range(16)]
    rgbs = [synth_gpu.he_slide(2048, 2048, seed=7300 + i, background=0.4, device="cuda") for i in range(16)]
    truth = [synth_gpu.tissue_mask(2048, 2048, seed=7300 + i, background=0.4) for i in range(16)]
    labs_p = [torch.empty((2048, 2048), dtype=torch.int32, device="cuda") for _ in rgbs]
    labs_g = [torch.empty((2048, 2048), dtype=torch.int32, device="cuda") for _ in rgbs]
    pixels = 16 * 2048 * 2048

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    def mean(rows, k):
        return round(sum(r[k] for r in rows) / len(rows), 5)

    dt_p = timed(lambda: ctx.segment_batch(rgbs, base, report=False, labels=labs_p))
    out_roi = {}
    g_paper = None
    for fs in ("roi", "learned"):
        p = dict(base, gate_rule="differ", gate_features=fs)
        Xs, ts = [], []
        for rgb, roi in zip(train, train_roi):
            X, t = gate.roi_samples(ctx, rgb, roi, p)
            Xs.append(X)
            ts.append(t)
        X, t = torch.cat(Xs), torch.cat(ts)
        _, w = gate.train(ctx, X, t, epochs=20, batch=4096, seed=0)
        z, _ = ctx.mlp_forward(X, w, 0.0)
        acc = float(((z >= 0) == t.bool()).float().mean().item())
        holder = {}

        def gated():
            holder["g"] = ctx.segment_gated(rgbs, p, w, 0.0, labels=labs_g, report=False)[3]

        dt_g = timed(gated)
        g = holder["g"]
        K = g.numel() // len(rgbs)
        if fs == "roi":
            g_paper = g.clone()
        sc_p, sc_g, brs = [], [], []
        for i in range(16):
            gi = g[i * K:(i + 1) * K]
            sc_p.append(gate.roi_scores(gate.roi_mask(labs_p[i], gi), truth[i]))
            sc_g.append(gate.roi_scores(gate.roi_mask(labs_g[i], gi), truth[i]))
            brs.append(gate.boundary_recall(ctx, labs_p[i], labs_g[i]))
        out_roi[fs] = {
            "features": ("the paper's four: absolute and comparative brightness, extra- and intra-region "
                         "dissimilarity" if fs == "roi" else "the learned gate's sixteen"),
            "train_accuracy": round(acc, 4), "samples": int(X.shape[0]),
            "positive_rate": round(float(t.float().mean().item()), 4),
            "MPixel/s": round(pixels / dt_g / 1e6, 3), "ms": round(dt_g * 1e3, 3), "speedup": round(dt_p / dt_g, 4),
            "br_vs_plain": round(sum(brs) / len(brs), 5), "marked_roi": round(float(g.float().mean().item()), 4),
            "plain_roi": {k: mean(sc_p, k) for k in ("precision", "recall", "f1")},
            "gated_roi": {k: mean(sc_g, k) for k in ("precision", "recall", "f1")}}
        print("bench: roi classifier on %s features: accuracy %.4f, %.2fx, BR %.4f"
              % (fs, acc, dt_p / dt_g, out_roi[fs]["br_vs_plain"]), file=sys.stderr, flush=True)

    # the learned boundary-recall gate at the paper gate's boundary recall
    pb = dict(base, gate_rule="both", gate_features="learned")
    Xb, tb = gate.training_set(ctx, train, pb)
    _, wb = gate.train(ctx, Xb, tb, epochs=20, batch=4096, seed=0)
    target = out_roi["roi"]["br_vs_plain"]
    K = g_paper.numel() // len(rgbs)
    out_br = []
    for th in (1e9, 4.0, 3.0, 2.0, 1.5, 1.0, 0.5, 0.0, -0.5, -1.0, -2.0, -1e9):
        ctx.segment_gated(rgbs, pb, wb, th, labels=labs_g, report=False)
        br = sum(gate.boundary_recall(ctx, a, b) for a, b in zip(labs_p, labs_g)) / len(rgbs)
        holder = {}

        def gated_br():
            holder["g"] = ctx.segment_gated(rgbs, pb, wb, th, labels=labs_g, report=False)[3]

        dt_b = timed(gated_br)
        sc_b = [gate.roi_scores(gate.roi_mask(labs_g[i], g_paper[i * K:(i + 1) * K]), truth[i]) for i in range(16)]
        out_br.append({"thresh": th, "br_vs_plain": round(br, 5), "MPixel/s": round(pixels / dt_b / 1e6, 3),
                       "speedup": round(dt_p / dt_b, 4), "marked": round(float(holder["g"].float().mean().item()), 4),
                       "roi_with_paper_classes": {k: mean(sc_b, k) for k in ("precision", "recall", "f1")}})
        # the thresholds that bracket the paper gate's boundary recall
        if br >= target:
            break
    out_br = {"rule": "both", "gate_level": 1, "points": out_br[-2:] if len(out_br) > 1 else out_br,
              "note": "thresholds from 1e9 (nothing refined past the gate) down to the first whose mean boundary "
                      "recall on the 16 tiles reaches the paper gate's; the last two bracket it"}
    out = {
        "metric": METRIC, "value": round(pixels / dt_p / 1e6, 3), "unit": "MPixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt_p * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "16 RGB uint8 2048x2048 synthetic H&E tiles (40% background) in one launch, "
                               "K=4096 each, three levels 16|8,4|2,1; region of interest = tissue",
                   "pixels": pixels, "path": "plain"},
        "roi": {"paper_gate": out_roi["roi"], "sixteen_feature_gate": out_roi["learned"],
                "learned_br_gate_at_equal_br": out_br,
                "note": "rule differ at level 2 (pairs across the predicted ROI border refine); pixel precision / "
                        "recall / F1 of the ROI masks against the generator's tissue mask, mean over the 16 "
                        "held-out tiles; the paper reports precision 0.816 and F1 0.898 on NLST (context only)"},
    }
    ctx.close()
    out["device"] = device_facts()
    print(json.dumps(out), flush=True)


def bench_he(args):
    """H&E workloads: the 65536 x 49152 slide (default), the 32768^2 slide,
    or one 4096^2 or 8192^2 image; plain, and gated (the 65536 x 49152 slide
    unless --no-gated; the 4096^2 image and the 32768^2 slide with
    --gated)."""
    import torch
    from paper_1704_02083_amd import rapid, synth_gpu
    _, p, desc = workload(args.workload)
    slide = args.workload in ("slide", "slide65k")
    gated = args.gated or (args.workload == "slide65k" and not args.no_gated and args.grain == 1)
    if args.grain > 1:
        # drop the stages finer than the grain (levels keep their factor)
        lv = [(f, [b for b in st if b * f >= args.grain]) for f, st in p["levels"]]
        p = dict(p, levels=[(f, st) for f, st in lv if st])
        desc += ", grain %d (stages of effective block size >= %d only)" % (args.grain, args.grain)
        if args.gated:
            raise SystemExit("--grain applies to the plain path only")
    if gated and args.workload == "he8192":
        raise SystemExit("--gated applies to he4096, slide and slide65k")
    ctx = rapid.Context(0, timing=True, autotune=not args.no_autotune)
    if slide:
        W, H, seed = (32768, 32768, 4) if args.workload == "slide" else (65536, 49152, 5)
        rgb = synth_gpu.he_slide(W, H, seed=seed, background=0.4, device="cuda", band=1024)
        labels = torch.empty((H, W), dtype=torch.int32, device="cuda")
        lay = rapid.tile_layout(W, H, 2048, 64, 32)

        def run():
            ctx.segment_slide(rgb, p, tile=2048, halo=64, cell=32, labels=labels)
    else:
        W = H = 8192 if args.workload == "he8192" else 4096
        rgb = synth_gpu.he_slide(W, H, seed=3, background=0.3, device="cuda")
        labels = torch.empty((H, W), dtype=torch.int32, device="cuda")

        def run():
            ctx.segment(rgb, p, labels=labels, report=False)
    torch.cuda.synchronize()
    print("bench: %s generated" % args.workload, file=sys.stderr, flush=True)

    dt, ref_ms, tune_call = timed_steps(ctx, run, args)
    print("bench: plain, %d steps of %.3f ms" % (args.steps, dt * 1e3), file=sys.stderr, flush=True)
    tm = ctx.last_timings()
    shape = {"threads": tm["threads"], "stats_lds": tm["stats_lds"], "pyramid_in_launch": tm["pyramid"],
             "workgroups_per_image": tm["workgroups"], "autotuned": not args.no_autotune}
    # one image spread over a cooperative launch runs the k_refine_mc kernel
    kname = "k_refine_mc" if tm["workgroups"] > 1 else "k_refine"
    plain = labels.clone()
    # per-stage counters of the same deterministic work, from one untimed call
    if slide:
        _, reps = ctx.segment_slide(rgb, p, tile=2048, halo=64, cell=32, labels=labels, report=True)
        alg, alg_w = tiles_alg_bytes(W, H, lay, reps), tiles_alg_bytes(W, H, lay, reps, stage_bytes_window)
    else:
        _, r = ctx.segment(rgb, p, labels=labels, report=True)
        py = bool(tm["pyramid"])
        alg = refine_alg_bytes([rgb], [r], pyramid=py)
        alg_w = refine_alg_bytes([rgb], [r], stage_bytes_window, pyramid=py)
    traffic = profile_traffic(kname, args.workload + ("_grain%d" % args.grain if args.grain > 1 else ""),
                              kernel_source_hash())
    out = {
        "metric": METRIC, "value": round(W * H / dt / 1e6, 3), "unit": "MPixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": desc, "pixels": W * H, "path": "plain"},
        "roofline": roofline(kname, alg, alg_w, ref_ms, traffic),
        "launch_shape": shape,
        "autotune_call": tune_call,
    }
    if gated:
        out["gated"] = bench_gated(args, ctx, rgb, labels, plain, W, H, dt)
    if args.reuse_baseline:
        if args.workload != "he4096":
            raise SystemExit("--reuse-baseline applies to he4096")
        out["reuse"] = bench_reuse(ctx, rgb, p, plain)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        if slide:
            out["cpu_baseline"] = cpu_baseline_tiles(rgb, W, H, p, lay)
        else:
            out["cpu_baseline"] = cpu_baseline([rgb.cpu().numpy()], p, 1)
    ctx.close()
    out["device"] = device_facts()
    print(json.dumps(out), flush=True)


def bench_reuse(ctx, rgb, p, plain, reps: int = 3):
    """Level by level through the state API: statistics carried from level
    to level (Sec. 3.2) against the same run with the statistics recounted
    from the pixels at every level (labels mapped to pixels and back), as
    multi-scale CTFTPS recomputes them.  The sums are exact either way, so
    both must give the plain labels."""
    import torch
    n_levels = len(p["levels"])

    def run(recount):
        st = ctx.state(rgb, p)
        for l in range(n_levels):
            if recount and l > 0:
                lab, _ = st.export()
                st.import_(l, lab, None)
            st.refine_level(l, report=False)
        lab, _ = st.export()
        st.close()
        return lab

    out = {}
    for name, recount in (("reuse", False), ("recount", True)):
        run(recount)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            lab = run(recount)
        torch.cuda.synchronize()
        out[name + "_ms"] = round((time.perf_counter() - t0) * 1e3 / reps, 3)
        out[name + "_identical_to_plain"] = bool((lab == plain).all().item())
    out["recount_over_reuse"] = round(out["recount_ms"] / out["reuse_ms"], 4)
    return out


if __name__ == "__main__":
    main()
