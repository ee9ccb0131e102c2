"""Device math of the coefficient path, compiled for the host and checked on
the CPU: the bounded-argument sin/cos and the root finder (the exact code the
root kernel runs), against 30-50 digit arithmetic; and the autotuner's
on-disk cache (write, read back, damaged files)."""
import math
import os
import shutil
import subprocess

import mpmath as mp
import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("host") / "device_math_harness")
    cmd = [HIPCC, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
           "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2608_16208_amd", "csrc"),
           "-o", exe, os.path.join(ROOT, "tests", "host", "device_math_harness.cpp")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    return exe


@pytest.mark.parametrize("mode", ["sincos", "sincosm"])
def test_sincos_bounded_accuracy(harness, mode):
    """sincos_bounded and sincos_moderate (the quadrant from a 32-bit
    conversion) against 50-digit sin and cos, negative arguments included."""
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.uniform(-100, 100, 400), rng.uniform(-1e-3, 1e-3, 50),
                         np.array([0.0, math.pi / 4, math.pi / 2, math.pi, 3 * math.pi / 2,
                                   1e-300, -2.5, -3 * math.pi / 4, 1000.0, 12345.678])])
    out = subprocess.run([harness, mode], input="\n".join(repr(float(x)) for x in xs),
                         capture_output=True, text=True).stdout.split()
    got = np.array(out, dtype=float).reshape(-1, 2)
    mp.mp.dps = 50
    for x, (s, c) in zip(xs, got):
        rs, rc = mp.sin(mp.mpf(float(x))), mp.cos(mp.mpf(float(x)))
        assert abs(s - float(rs)) <= 3e-16 * max(1e-300, abs(float(rs))) + 2.3e-16 * (abs(x) > 1e-3)
        assert abs(c - float(rc)) <= 3.3e-16


@pytest.mark.parametrize("cfgi", [2, 3])
def test_root_finder_on_host(harness, cfgi):
    """Roots from the root kernel's code zero rho^2 to 1e-13 b (30-digit check)."""
    cfg = workloads.config(cfgi)
    M, a = cfg["M"], cfg["amp"]
    t, j, ts = workloads.sample_pairs(cfg["n_panels"], M, 60, seed=700 + cfgi)
    inp = (f"{M} {cfg['k']} {a.shape[0]} {a.shape[1] - 1}\n"
           + " ".join(repr(float(v)) for v in a.ravel()) + f"\n{len(t)}\n"
           + "\n".join(f"{float(t[i])!r} {int(j[i])} {float(ts[i])!r}" for i in range(len(t))))
    out = subprocess.run([harness], input=inp, capture_output=True, text=True).stdout.split()
    res = np.array(out, dtype=float).reshape(-1, 7)
    mp.mp.dps = 30

    def r_mp(tt, th):
        R = 1 + sum(mp.mpf(float(a[l - 1, m])) * mp.sin(l * tt) * mp.cos(m * th)
                    for l in range(1, a.shape[0] + 1) for m in range(a.shape[1]) if a[l - 1, m])
        return [R * mp.sin(tt) * mp.cos(th), R * mp.sin(tt) * mp.sin(th), R * mp.cos(tt)]

    checked = 0
    for i in range(len(t)):
        u, b, st, eb, omq, sh, ch = res[i]
        # the root-only values the record carries for the coefficient passes:
        # e^{-b} and 1 - e^{-b} to a few ulp, relative; the half offset of the
        # root from the nearest point of the 2M-point grid, step pi/M
        bm = mp.mpf(float(b))
        assert abs(eb - float(mp.exp(-bm))) <= 4e-16 * float(mp.exp(-bm)), (i, b)
        assert abs(omq - float(-mp.expm1(-bm))) <= 4e-16 * float(-mp.expm1(-bm)), (i, b)
        um = mp.mpf(float(u))
        qu = int(round(float(u) * M / math.pi))
        half = (um - qu * mp.pi / M) / 2
        assert abs(half) <= mp.pi / (4 * M) * (1 + 1e-12)
        assert abs(sh - float(mp.sin(half))) <= 1e-15 and abs(ch - float(mp.cos(half))) <= 1e-15, i
        if int(st) & (2 | 16):
            continue
        th = mp.pi * int(j[i]) / M
        p0 = r_mp(mp.mpf(float(t[i])), th)
        f = lambda zz: sum((x - y) ** 2 for x, y in zip(r_mp(mp.mpf(float(ts[i])), zz), p0))
        z = th + mp.mpf(u) + 1j * mp.mpf(b)
        assert b > 0
        assert abs(f(z) / mp.diff(f, z)) <= 1e-13 * b, (i, b)
        checked += 1
    assert checked >= 40


def test_tuning_cache_round_trip_and_damaged_files(harness, tmp_path):
    path = str(tmp_path / "tune.json")
    out = subprocess.run([harness, "tunecache", path], capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.split("\n")
    assert lines[0] == "2"
    assert lines[1] == "gfx950 x256|64|f64|2|16|4|0|12.5"
    assert lines[2] == "gfx950 x256|128|f32|4|8|2|1|0.25"
    assert lines[3] == "4 0"                      # hit on (M, precision), miss on the other precision
    import json
    doc = json.load(open(path))                   # the file is plain JSON
    assert doc["format"] == "ffbie-tuning-cache" and len(doc["entries"]) == 2

    def read(text):
        with open(path, "w") as fh:
            fh.write(text)
        r = subprocess.run([harness, "tunecache", path, "read"], capture_output=True, text=True)
        return r.stdout.split("\n")[0]

    assert read(json.dumps(doc)) == "2"           # re-serialised by another writer: still read
    assert read('{"format": "something-else", "entries": []}') == "0"
    assert read(json.dumps(doc)[:-20]) == "0"     # truncated
    doc["entries"][0]["extra"] = 1
    assert read(json.dumps(doc)) == "0"           # unknown key: the whole file is ignored
