"""Summarise rocprofv3 counter and trace runs of bench.py into the HBM traffic
record that bench.py reports (``profiles/sep_passes_<workload>_traffic.json``).

  python counters.py --fetch D1 --write D2 --trace D3 \\
      --calib-fetch D4 --calib-write D5 --workload vol512

D1/D2: ``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` output directories
of the same bench.py command; D3: its ``--kernel-trace --stats`` directory;
D4/D5: FETCH_SIZE / WRITE_SIZE of ``bench.py --config calibrate`` (a reslice of
a 1 GiB float32 stack: 1 GiB read and 1 GiB written per launch).  The counters
give KiB per dispatch; each is scaled by the factor that makes the calibration
kernel's reading equal its known traffic.  A second kernel of known size, the
first kernel of the bench run (ψ^0 from two uint16 views: 4 B read and 4 B
written per voxel), is reported beside it as a cross-check, and so is the
calibration run's plain copy of the same 1 GiB.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import statistics

ROOT = os.path.dirname(os.path.abspath(__file__))


def _rows(d, name):
    files = glob.glob(os.path.join(d, "**", f"*{name}.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{name}.csv under {d}")
    out = []
    for f in files:
        with open(f, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


def per_kernel(d, counter):
    """Mean counter value (per dispatch) of every kernel name in a --pmc run."""
    vals = {}
    for r in _rows(d, "counter_collection"):
        if r.get("Counter_Name") != counter:
            continue
        vals.setdefault(r["Kernel_Name"], {}).setdefault(r["Dispatch_Id"], 0.0)
        vals[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return {k: statistics.fmean(v.values()) for k, v in vals.items()}


def trace_stats(d):
    out = {}
    for r in _rows(d, "kernel_stats"):
        out[r["Name"]] = {"calls": int(r["Calls"]), "avg_us": float(r["AverageNs"]) / 1e3}
    return out


def main():
    ap = argparse.ArgumentParser()
    for k in ("fetch", "write", "trace", "calib_fetch", "calib_write"):
        ap.add_argument("--" + k.replace("_", "-"), required=True)
    ap.add_argument("--workload", default="vol512")
    ap.add_argument("--voxels", type=int, default=512 ** 3)
    ap.add_argument("--command", action="append", default=[], help="commands that made the runs (recorded)")
    a = ap.parse_args()
    import bench

    kib = 1024.0
    cal_bytes = 1024 ** 3
    cf, cw = per_kernel(a.calib_fetch, "FETCH_SIZE"), per_kernel(a.calib_write, "WRITE_SIZE")
    ck = [k for k in cf if "stage_kernel" in k]
    if len(ck) != 1:
        raise SystemExit(f"calibration kernel not found among {list(cf)}")
    fetch_factor = cal_bytes / (cf[ck[0]] * kib)
    write_factor = cal_bytes / (cw[ck[0]] * kib)
    fetch, write, trace = per_kernel(a.fetch, "FETCH_SIZE"), per_kernel(a.write, "WRITE_SIZE"), trace_stats(a.trace)
    kernels = {}
    for k in fetch:
        if k not in write:
            continue
        fb, wb = fetch[k] * kib * fetch_factor, write[k] * kib * write_factor
        t = trace.get(k, {})
        kernels[k] = {"fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb,
                      "trace_calls": t.get("calls", 0), "trace_avg_us": t.get("avg_us")}
    # cross-check: the run's ψ^0 kernel reads 2 uint16 views and writes a float32 mean
    sv = [k for k in kernels if "stage_views_kernel" in k]
    check = None
    if sv:
        kv = kernels[sv[0]]
        check = {"kernel": sv[0], "expected_read": 4 * a.voxels, "expected_write": 4 * a.voxels,
                 "read_ratio": kv["fetch_bytes"] / (4 * a.voxels), "write_ratio": kv["write_bytes"] / (4 * a.voxels)}
    # second cross-check from the calibration run itself: the plain copy of the
    # same 1 GiB (probe_copy_kernel), scaled by the reslice's factors
    copy_check = None
    pc = [k for k in cf if "probe_copy_kernel" in k and k in cw]
    if pc:
        copy_check = {"kernel": pc[0], "read_ratio": cf[pc[0]] * kib * fetch_factor / cal_bytes,
                      "write_ratio": cw[pc[0]] * kib * write_factor / cal_bytes}
    rec = {
        "code_sha256": {f: bench.pass_code_hash(f) for f in bench.PASS_SOURCES},
        "calibration": {"kernel": ck[0], "bytes_read": cal_bytes, "bytes_written": cal_bytes,
                        "fetch_kib": cf[ck[0]], "write_kib": cw[ck[0]]},
        "fetch_factor": fetch_factor, "write_factor": write_factor,
        "cross_check": check,
        "copy_check": copy_check,
        "kernels": kernels,
        "commands": a.command,
    }
    path = os.path.join(ROOT, "profiles", f"sep_passes_{a.workload}_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"wrote {path}")
    print(f"calibration: {ck[0]}: FETCH x{fetch_factor:.3f}, WRITE x{write_factor:.3f}")
    if check:
        print(f"cross-check {check['kernel'][:60]}: read {check['read_ratio']:.3f}, write {check['write_ratio']:.3f} "
              f"of the known traffic")
    if copy_check:
        print(f"copy check {copy_check['kernel'][:60]}: read {copy_check['read_ratio']:.3f}, "
              f"write {copy_check['write_ratio']:.3f} of the known traffic")
    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["trace_calls"])[:8]:
        print(f"- `{k[:70]}`: {v['fetch_bytes'] / 1e9:.3f} GB read + {v['write_bytes'] / 1e9:.3f} GB written "
              f"= {v['traffic_bytes'] / 1e9:.3f} GB per launch; {v['trace_calls']} calls, "
              f"{v['trace_avg_us']} us average")


if __name__ == "__main__":
    main()
