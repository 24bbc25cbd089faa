"""Host-side logic of bench.py (no GPU): the work model behind the roofline
entry, the choice of bound, the traffic record's guards and the one-GPU rule."""
import json
import os
import subprocess
import sys

import pytest

import bench
from synthetic import CONFIGS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_step_work_vol512():
    """Per voxel: forward reads ψ once and, per view, φ (uint16) and writes r;
    backward reads r per view and reads + writes ψ; flops 2·(K + K) per view."""
    spec = CONFIGS["vol512"]
    vox = spec.n_planes * spec.n_z * spec.n_x
    b, f, fv, fm = bench.step_work_split(spec, "forward", vox, 1)
    assert b == vox * (4 + (2 + 4) * 2) and f == vox * 2 * 2 * 62 and fv == 0 and fm == f
    b, f, _, _ = bench.step_work_split(spec, "backward", vox, 1)
    assert b == vox * (8 + 4 * 2)
    b2, f2, _, _ = bench.step_work_split(spec, "backward", vox, 2)     # views over 2 launches
    assert b2 == vox * (4 * 2 + 8 * 2) / 2 and f2 == f / 2
    b, f, _, fm = bench.step_work_split(spec, "forward", vox, 1, general=True)
    assert b == vox * (4 + 8 * 2) and f == fm == vox * 2 * 2 * 31 * 31


def _kinds(ms):
    spec = CONFIGS["vol512"]
    vox = spec.n_planes * spec.n_z * spec.n_x
    out = {}
    for kind in ("forward", "backward"):
        b, f, fv, fm = bench.step_work_split(spec, kind, vox, 1)
        out[kind] = dict(launches=10, avg_ms=ms[kind], bytes=b, flops=f, flops_valu=fv, flops_mfma=fm)
    return spec, out


def test_roofline_bound_and_fraction():
    spec, kinds = _kinds({"forward": 0.50, "backward": 0.55})
    r = bench.roofline(spec, kinds, variant=True)
    assert r["bound"] == "hbm" and r["kernel"].startswith("backward")
    assert r["achieved"] == pytest.approx(kinds["backward"]["bytes"] / 0.55e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["traffic"] is None                  # variants were not counted
    assert r["floor_ms"]["alu"] == 0.0


def test_traffic_record_guard():
    """The committed counter record is used only while its kernel-code hash
    matches; a record for another workload name does not exist."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "sep_passes_vol512_traffic.json")))
    got = bench.measured_traffic("vol512", "backward")
    same = rec.get("code_sha256", {}).get("sep") == bench.pass_code_hash("sep")
    assert (got is not None) == same
    if got is not None:
        assert got["bytes"] > 0 and "backward" in got["instance"]
    assert bench.measured_traffic("no_such_workload", "backward") is None


def test_kernel_code_hash_ignores_comments(tmp_path):
    a = tmp_path / "a.hpp"
    b = tmp_path / "b.hpp"
    c = tmp_path / "c.hpp"
    a.write_text("int f(int x) {  // doubles\n  return 2 * x; /* note */\n}\n")
    b.write_text("// another remark\nint f(int x) {\n  return 2 * x;\n}\n")
    c.write_text("int f(int x) {\n  return 3 * x;\n}\n")
    assert bench.kernel_code_hash(a) == bench.kernel_code_hash(b)
    assert bench.kernel_code_hash(a) != bench.kernel_code_hash(c)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stdout + p.stderr


def test_cpu_baseline_is_bounded():
    """The oracle leg times one plane per worker process (as many workers as
    the host gives, at most 16); planes larger than 512×512 get fewer
    iterations so that the leg stays a few seconds."""
    import numpy as np

    from synthetic import VolumeSpec

    spec = VolumeSpec("tiny", 3, 24, 20, 5, (1.0, 2.0), (0, 90), 4, "u16", 3, "simultaneous", seed=9)
    rng = np.random.default_rng(0)
    vol = {"stacks": [rng.integers(90, 200, (24, 3, 20)).astype(np.uint16) for _ in range(2)],
           "psfs": [np.full((5, 5), 1 / 25, dtype=np.float32)] * 2}
    out = bench.cpu_baseline(spec, vol, spec.iters)
    assert out["kind"] == "oracle" and out["value"] > 0 and "all 3 iterations" in out["sample"]
    assert out["cores"] == min(3, bench.host_cores())   # 3 planes: at most 3 workers
    wide = VolumeSpec("wide", 1, 1024, 1024, 3, (1.0, 2.0), (0, 90), 4, "u16", 10, "simultaneous", seed=9)
    vol = {"stacks": [rng.integers(90, 200, (1024, 1, 1024)).astype(np.uint16) for _ in range(2)],
           "psfs": [np.full((3, 3), 1 / 9, dtype=np.float32)] * 2}
    out = bench.cpu_baseline(wide, vol, wide.iters)
    assert "2 of 10 iterations" in out["sample"]
