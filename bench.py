"""Benchmark of the RAPID refinement sweep on one MI355X.

A step is one whole segmentation of the batch (block-sum pyramid, grid,
every stage and sweep of the refinement, pixel labels written) with the
images already resident in HBM.  The default workload is the batched one:
200 synthetic RGB uint8 images (100 of 481x321 and 100 of 321x481, Voronoi
mosaics of 30..120 regions with linear colour gradients and N(0, 6^2) noise),
400 superpixels each, one level with block sizes 16, 8, 4, 2, 1.

Prints one JSON line: throughput in MPixel/s, the roofline of the dominant
kernel (the refinement kernel, HBM-bound by design: there is no dense
contraction), and the CPU oracle timed on a bounded sample of the same
workload on this host.
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
    h = hashlib.sha256()
    for f in ("rapid_kernels.hip", "rapid_internal.h"):
        with open(os.path.join(ROOT, "paper_1704_02083_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(name: str):
    from paper_1704_02083_amd import params, synth
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


def refine_alg_bytes(imgs, reports) -> float:
    """Algorithmic bytes of one refinement launch: per stage the label map is
    written once and read once by the boundary scan (8 B per block); every
    block visit reads its 3x3 label window (36 B) and its colour sum (8 B
    packed, 3 B at B = 1); every commit writes a label (4 B) and reads the
    sum again; the final pixel labels are written once (4 B per pixel).
    Per-superpixel statistics stay on chip (LDS) and count zero."""
    total = 0
    for img, rep in zip(imgs, reports):
        H, W = img.shape[:2]
        total += 4 * W * H
        for r in rep:
            B = r["block"]
            nb = -(-W // B) * -(-H // B)
            sb = 3 if B == 1 else 8
            total += 8 * nb + r["active"] * (36 + sb) + r["commits"] * (4 + sb)
    return float(total)


def block_sums_alg_bytes(imgs, p) -> float:
    total = 0
    for img in imgs:
        H, W = img.shape[:2]
        for f, st in p["levels"]:
            for b in st:
                B = b * f
                if B >= 2:
                    total += 3 * W * H + 8 * (-(-W // B) * -(-H // B))
    return float(total)


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
    return {"value": round(px / dt / 1e6, 4), "unit": "MPixel/s", "cores": 1, "kind": "oracle",
            "sample": "%d of the %d images (%d px), single-threaded, %.1f s" % (n, len(imgs), px, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch", choices=["batch", "single256"])
    ap.add_argument("--cpu-sample", type=int, default=80)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy three times (scales the HBM "
                         "byte counters of rocprofv3 --pmc)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the refinement path runs on a single MI355X "
              "(multi-GPU sharding is not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1704_02083_amd import rapid

    if args.copy_calibration:
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "launches": 3}), flush=True)
        return

    imgs, p, desc = workload(args.workload)
    print("bench: workload %s, %d images generated" % (args.workload, len(imgs)), file=sys.stderr,
          flush=True)
    rgbs = [torch.from_numpy(im).cuda() for im in imgs]
    labels = [torch.empty(im.shape[:2], dtype=torch.int32, device="cuda") for im in imgs]
    ctx = rapid.Context(0, timing=True)
    pixels = sum(im.shape[0] * im.shape[1] for im in imgs)

    def step():
        if len(rgbs) == 1:
            ctx.segment(rgbs[0], p, labels=labels[0], report=False)
        else:
            ctx.segment_batch(rgbs, p, labels=labels, report=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    refine_ms, sums_ms = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        t = ctx.last_timings()
        refine_ms.append(t["refine_ms"])
        sums_ms.append(t["block_sums_ms"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print("bench: timed %d steps in %.3f s" % (args.steps, dt), file=sys.stderr, flush=True)

    # counters of the same (deterministic) work, from one untimed call
    if len(rgbs) == 1:
        _, r = ctx.segment(rgbs[0], p, labels=labels[0], report=True)
        reps = [r]
    else:
        _, reps = ctx.segment_batch(rgbs, p, labels=labels, report=True)
    ms_step = dt * 1e3 / args.steps
    avg_refine = sum(refine_ms) / len(refine_ms)
    alg = refine_alg_bytes(imgs, reps)
    achieved = alg / (avg_refine * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    traffic = profile_traffic("k_refine", args.workload, src_hash)
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
                   "superpixels_per_image": p["K"], "path": "plain"},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_refine",
            "achieved": round(achieved, 3),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 6),
            "traffic": traffic,
            "alg_bytes_per_launch": alg,
            "avg_launch_ms": round(avg_refine, 4),
            "block_sums_ms": round(sum(sums_ms) / len(sums_ms), 4),
            "source_hash": src_hash,
        },
    }
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(imgs, p, args.cpu_sample)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
