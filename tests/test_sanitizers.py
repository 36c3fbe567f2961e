"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
sanitized build runs every entry point (plain and gated segmentation under
each pair rule, merge on underflow, the FIFO schedule, features, energies,
proposals) in a fresh process; any report aborts it."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import numpy as np
import oracle
from paper_1704_02083_amd import params, synth
img = synth.voronoi_blur(96, 64, regions=8, seed=3)
p = params.default_params(96, 64, 12, levels=params.THREE_LEVEL, gate_level=1)
K = oracle.n_superpixels(96, 64, p)
gate = (np.random.default_rng(1).random(K) < 0.5).astype(np.uint8)
for rule in ("either", "both", "differ"):
    oracle.segment(img, dict(p, gate_rule=rule), gate=gate, debug=True)
lab, st, rep, inv, mov = oracle.segment(img, p, debug=True, track=True)
oracle.segment(img, dict(p, min_size=100, merge=True), debug=True)
oracle.segment(img, p, debug=True, shuffle_seed=7)
oracle.segment_fifo(img, dict(p, gate_level=-1), debug=True)
gx, gy = oracle.grid(96, 64, 12)
oracle.features(img, lab, 1, st, mov, gx, gy)
oracle.energy(img, p, lab)
oracle.merge_cost(img, p, lab, K, 0, 1)
oracle.block_energy(img, p, lab, K, 1, 5, 5, int(lab[5, 6]))
oracle.propose_class(img, p, lab, K, 1, 0)
print("sanitized ok")
'''


def test_oracle_clean_under_asan_ubsan(tmp_path):
    try:
        asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    except (OSError, subprocess.CalledProcessError):
        pytest.skip("gcc not available")
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan not available")
    lib = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "sanitized ok" in r.stdout, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]


HOST_SCRIPT = r'''
import ctypes as C
from paper_1704_02083_amd import rapid, params
assert rapid.check_params(481, 321, params.config2(481, 321)) == 400
assert rapid.check_params(4096, 4096, params.config3()) == 16384
assert rapid.check_params(2048, 2048, dict(params.gated(2048, 2048, 4096), merge=True)) > 0
lut = (C.c_uint32 * 8)()
assert rapid._lib.rapid_simple_lut(lut) == 0
gx, gy = C.c_int32(), C.c_int32()
assert rapid._lib.rapid_grid(481, 321, 400, C.byref(gx), C.byref(gy)) == 0
for bad in (dict(params.config1(), frac_bits=9), dict(params.config1(), levels=[(1, [8, 16])]),
            dict(params.config1(), K=100000), dict(params.config1(), w_pos=1 << 40)):
    try:
        rapid.check_params(256, 256, bad)
        raise SystemExit("accepted a bad parameter set")
    except rapid.RapidError as e:
        assert e.code == -1
assert rapid.slide_tiles(65536, 49152, 2048, 64, 32) == 768
for c in range(-6, 1):
    rapid._lib.rapid_status_str(c)
print("host ok")
'''


def test_host_library_clean_under_asan_ubsan(tmp_path):
    """The library's host code (validation, grid, simple-point table, slide
    tiling) built with AddressSanitizer and UndefinedBehaviorSanitizer on the
    host side only, driven through its host-only entry points."""
    from paper_1704_02083_amd import build as b
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    rt = subprocess.run([hipcc, "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    asan = rt.stdout.strip()
    if rt.returncode != 0 or not os.path.isabs(asan) or not os.path.exists(asan):
        import glob
        found = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        if not found:
            pytest.skip("clang's ASan runtime not found")
        asan = found[0]
    lib = str(tmp_path / "librapid_san.so")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", b.CSRC, "-o", lib] + \
        [os.path.join(b.CSRC, s) for s in b.SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, RAPID_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", HOST_SCRIPT], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "host ok" in r.stdout, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
