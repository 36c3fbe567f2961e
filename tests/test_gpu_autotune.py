"""The autotuner and the launch shapes it chooses between: every shape
(workgroup size; per-superpixel state in LDS, only the means records in LDS,
or all in global memory; pyramid inside the launch or not) gives the same
labels, and tuned choices persist in the cache file."""
import os

import numpy as np
import pytest

import oracle
from paper_1704_02083_amd import params, synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _batch(n):
    import torch
    imgs = synth.batch_images(n)
    return imgs, [torch.from_numpy(im).cuda() for im in imgs]


def test_every_launch_shape_same_labels(gpu_lib):
    """130 images (enough for the in-launch pyramid): all 24 shapes give the
    labels of the default shape; image 7 also equals the oracle."""
    import torch
    imgs, rgbs = _batch(130)
    p = params.config2(481, 321)
    c = gpu_lib.Context(0)
    ref, ref_rep = c.segment_batch(rgbs, p)
    ref = [l.cpu().numpy() for l in ref]
    c.close()
    o, _, o_rep = oracle.segment(imgs[7], p)
    assert (ref[7] == o).all() and ref_rep[7] == o_rep
    old = os.environ.get("RAPID_SHAPE")
    try:
        for t in (256, 512, 1024):
            for lds in (1, 3, 2, 0):
                for py in (1, 0):
                    os.environ["RAPID_SHAPE"] = "%d,%d,%d" % (t, lds, py)
                    _say("case: shape threads %d stats_lds %d pyramid %d" % (t, lds, py))
                    c = gpu_lib.Context(0, timing=True)
                    labs, reps = c.segment_batch(rgbs, p)
                    torch.cuda.synchronize()
                    tm = c.last_timings()
                    assert (tm["threads"], tm["stats_lds"], tm["pyramid"]) == (t, lds, py)
                    for i in range(0, 130, 13):
                        assert (labs[i].cpu().numpy() == ref[i]).all(), (t, lds, py, i)
                        assert reps[i] == ref_rep[i]
                    c.close()
    finally:
        if old is None:
            os.environ.pop("RAPID_SHAPE", None)
        else:
            os.environ["RAPID_SHAPE"] = old


def test_autotune_chooses_and_caches(gpu_lib, tmp_path):
    import torch
    imgs, rgbs = _batch(130)
    p = params.config2(481, 321)
    c = gpu_lib.Context(0)
    ref, _ = c.segment_batch(rgbs, p, report=False)
    ref = [l.cpu().numpy() for l in ref]
    c.close()
    cache = str(tmp_path / "tune.json")
    _say("case: autotune, fresh cache")
    c = gpu_lib.Context(0, timing=True, autotune=True, autotune_cache=cache)
    labs, _ = c.segment_batch(rgbs, p, report=False)
    t1 = c.last_timings()
    assert t1["tuned"] == 1 and t1["threads"] in (256, 512, 1024)
    labs2, _ = c.segment_batch(rgbs, p, report=False)
    t2 = c.last_timings()
    assert t2["tuned"] == 0
    assert (t2["threads"], t2["stats_lds"], t2["pyramid"]) == (t1["threads"], t1["stats_lds"], t1["pyramid"])
    for a, b, r in zip(labs, labs2, ref):
        assert (a.cpu().numpy() == r).all() and (b.cpu().numpy() == r).all()
    c.close()
    txt = open(cache).read()
    assert '"rapid_autotune": 1' in txt and "n130_W481_H481_K" in txt
    _say("case: autotune, cache read back")
    c = gpu_lib.Context(0, timing=True, autotune=True, autotune_cache=cache)
    labs3, _ = c.segment_batch(rgbs, p, report=False)
    t3 = c.last_timings()
    assert t3["tuned"] == 0
    assert (t3["threads"], t3["stats_lds"], t3["pyramid"]) == (t1["threads"], t1["stats_lds"], t1["pyramid"])
    for a, r in zip(labs3, ref):
        assert (a.cpu().numpy() == r).all()
    c.close()
    # a cache written for another architecture is ignored
    open(cache, "w").write(txt.replace('"arch": "', '"arch": "other-'))
    c = gpu_lib.Context(0, timing=True, autotune=True, autotune_cache=cache)
    c.segment_batch(rgbs, p, report=False)
    assert c.last_timings()["tuned"] == 1
    c.close()
