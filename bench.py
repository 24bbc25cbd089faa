"""Throughput of plane-wise multi-view Richardson-Lucy deconvolution on one GPU.

One step = one whole deconvolution of the workload (reslice + convert the
uint16 observations, ψ^0, then every RL iteration) with the inputs already
resident in device memory.  Prints one JSON line (see the keys below).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config vol512]

--config mix times the batched form against plain per-volume calls;
--config vol1024x4 times the streamed form (host stacks, batches of planes);
--config grad256 times the differentiable form (forward, MSE, reverse sweep);
--config planes2048 times 64 planes of 2048x2048 (the per-plane rate of the
2048^3 size class).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
# fp32 vector FMA without packed instructions: 256 CUs × 4 SIMDs × 16 lanes ×
# 2 flop × 2.4 GHz (the library is built with packed FP32 disabled)
ALU_PEAK = 256 * 4 * 16 * 2 * 2.4e9
MFMA_F32_PEAK = 157.3e12     # dense FP32 matrix-core peak (the general K×K passes)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# the paper's own timings (GTX TITAN Black, FFT convolution, sizes padded by the
# PSF), Supplementary Table 1: context for the matching workloads, not a target
PAPER_CONTEXT = {
    "vol512": "GTX TITAN Black, 512^3 padded, 2 views, 10 iterations: 4.0 s "
              "(3.36e8 voxel-iterations/s), Supplementary Table 1",
    "planes2048": "GTX TITAN Black, 2048^3 padded, 2 views, 10 iterations: 152.3 s "
                  "(5.64e8 voxel-iterations/s), Supplementary Table 1",
    "vol2048": "GTX TITAN Black, 2048^3 padded, 2 views, 10 iterations, disk to disk: 152.3 s "
               "(5.64e8 voxel-iterations/s), Supplementary Table 1",
}

# per-pixel view weights (--pixel-weights): the backward pass also reads them
WEIGHT_PLANES = False


def step_work(spec, kind, vox, launches_per_iter, general=False):
    """(bytes, flops) of one launch; see step_work_split for the flop split."""
    b, f, _, _ = step_work_split(spec, kind, vox, launches_per_iter, general)
    return b, f


# PSF terms per view (--psf lowrank: a sum of this many rank-one terms), and
# the terms one launch runs (the library pairs them)
PSF_TERMS = 1
TERMS_PER_LAUNCH = 2


def step_work_split(spec, kind, vox, launches_per_iter, general=False):
    """Algorithmic bytes and flops of one forward / backward launch over
    ``vox`` voxels (a whole volume, or one batch of planes).

    Per voxel and view, a forward pass reads φ_v (as given: 2 bytes for
    uint16 observations; the general K×K passes read float32 staged copies),
    writes r_v and (once per launch) reads ψ; a backward pass reads r_v and
    (once per launch) reads and writes ψ.  Each view's two 1D passes cost
    2 · (kz + kx) flops (FMA = 2); a general K×K pass costs 2 · kz · kx; a PSF
    of R rank-one terms runs R pairs of 1D passes, two terms per launch, through
    a partial-sum plane.
    The library may split the V views of an iteration over several launches,
    so the work of one iteration on those voxels is divided by its launches.
    """
    V = spec.n_views
    k = spec.psf_k
    n = launches_per_iter
    R = PSF_TERMS
    if kind == "fused":
        # one launch per iteration: ψ in, every view's φ_v (as given), ψ' out;
        # the ratio planes stay on chip.  Both passes' 1D convolutions.
        phi = 2 if spec.obs_dtype == "u16" else 4
        b = 8 + phi * V
        f = V * 2 * 2 * (k + k)
        return vox * b / n, vox * f / n, 0.0, vox * f / n
    if R > 1 and not general:
        # L = ⌈R / 2⌉ launches per view and direction: every launch reads its
        # input (ψ forward, r_v backward), the partial sum crosses each launch
        # boundary (written, read), the last adds φ_v (float32) and r_v forward,
        # ψ in and ψ out backward: 4L + 8(L − 1) + 8 = 12L bytes per voxel and view
        L = -(-R // TERMS_PER_LAUNCH)
        b = 12 * L * V
    elif kind == "forward":
        phi = 2 if (spec.obs_dtype == "u16" and not general) else 4
        b = (phi + 4) * V + 4 * n
    else:
        b = (8 if WEIGHT_PLANES else 4) * V + 8 * n
    f = V * 2 * (k * k if general else PSF_TERMS * (k + k))
    # where the flops run: the separable passes do both the column (z) and the
    # row (x) convolution on the matrix cores, and so do the general K×K passes
    f_mfma = f
    f_valu = 0
    return vox * b / n, vox * f / n, vox * f_valu / n, vox * f_mfma / n


def kernel_code_hash(*paths):
    """sha256 of C++ sources with their comments removed and their whitespace
    collapsed: edits to comments keep it, any change to the code does not."""
    import hashlib
    import re

    parts = []
    for path in paths:
        text = open(path, encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        parts.append(" ".join(text.split()))
    return hashlib.sha256("\n".join(parts).encode()).hexdigest()


# the sources of the pass kernels whose counters the traffic record holds: the
# separable passes, and the fused iteration (which also includes the former)
PASS_SOURCES = {"sep": ("k_sep_impl.hpp",), "fused": ("k_sep_impl.hpp", "k_fused.hip")}


def pass_code_hash(family="sep"):
    return kernel_code_hash(*[os.path.join(ROOT, "paper_1503_07998_amd", "csrc", f) for f in PASS_SOURCES[family]])


def measured_traffic(name, kind):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (scaled by the factors a copy of known size
    gives), or None when the kernel code changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"sep_passes_{name}_traffic.json")
    family = "fused" if kind == "fused" else "sep"
    try:
        rec = json.load(open(path))
        h = pass_code_hash(family)
    except OSError:
        return None
    if rec.get("code_sha256", {}).get(family) != h:
        return None
    # the instance of the pass (plain, split-view or fused form) that ran most
    # often in the profiled bench run
    names = ("fused_kernel",) if kind == "fused" else (f"sep_{kind}_kernel", f"sep_{kind}_split_kernel")
    cands = [(k, v) for k, v in rec["kernels"].items() if any(n in k for n in names)]
    if not cands:
        return None
    k, v = max(cands, key=lambda kv: kv[1].get("trace_calls", 0))
    return {"bytes": v["traffic_bytes"], "instance": k}


def copy_rate_gbs(nbytes=1 << 30, reps=5):
    """The library's plain copy kernel over `nbytes` (read once, written once),
    timed with HIP events on the current stream: GB/s of read + written bytes."""
    import ctypes

    import torch

    from paper_1503_07998_amd import _native as N

    lib = N.lib()
    probe = lib.mvd_internal_stream_probe
    probe.restype = ctypes.c_int
    probe.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    h = ctypes.c_void_p(stream.cuda_stream)
    for _ in range(2):
        if probe(0, src.data_ptr(), dst.data_ptr(), nbytes, h) != 0:
            raise N.MvdError(N.MVD_ERR_LAUNCH, "copy probe failed")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        probe(0, src.data_ptr(), dst.data_ptr(), nbytes, h)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms / 1e3) / 1e9


def roofline(spec, kinds, general=False, variant=False):
    """Roofline entry of the kernel with the largest share of the step.

    ``variant`` marks a run whose passes are other kernel instances than the
    profiled default run (normalised or per-pixel-weighted back-projection):
    its HBM traffic has not been counted, so none is reported.

    The binding ceiling is the largest of the HBM time (algorithmic bytes at
    8 TB/s), the vector-ALU time (row-pass flops at 78.6 TFLOP/s) and the
    matrix-core time (column-pass or K×K flops at the 157.3 TFLOP/s FP32
    matrix peak); `achieved` is measured against that ceiling's peak."""
    dom = max(kinds, key=lambda k: kinds[k]["avg_ms"] * kinds[k]["launches"])
    kd = kinds[dom]
    sec = kd["avg_ms"] / 1e3
    times = {"hbm": kd["bytes"] / HBM_PEAK, "alu": kd["flops_valu"] / ALU_PEAK,
             "mfma": kd["flops_mfma"] / MFMA_F32_PEAK}
    bound = max(times, key=times.get)
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": kd["bytes"] / sec / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s"}
    elif bound == "alu":
        roof = {"bound": "alu", "achieved": kd["flops_valu"] / sec / 1e12, "peak": ALU_PEAK / 1e12,
                "unit": "TFLOP/s"}
    else:
        # useful flops only: banded Toeplitz operands also multiply zeros
        roof = {"bound": "mfma", "achieved": kd["flops_mfma"] / sec / 1e12, "peak": MFMA_F32_PEAK / 1e12,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    meas = None if general or variant else measured_traffic(spec.name, dom)
    roof["traffic"] = meas["bytes"] if meas else None
    if general:
        roof["kernel"] = f"{dom} pass (twod_{dom}_kernel, general {spec.psf_k}x{spec.psf_k})"
    elif meas:
        roof["kernel"] = f"{dom} pass ({meas['instance']})"
    elif dom == "fused":
        roof["kernel"] = f"fused iteration (fused_kernel, K={spec.psf_k})"
    else:
        roof["kernel"] = f"{dom} pass (sep_{dom} kernels, K={spec.psf_k})"
    roof["floor_ms"] = {k: v * 1e3 for k, v in times.items()}
    roof["hbm_frac_algorithmic"] = kd["bytes"] / sec / HBM_PEAK
    return roof


def launch_kinds(spec, tim, steps, vox, batches=1, general=False):
    """Per-kind launch statistics of ``steps`` timed runs (HIP events)."""
    kinds = {}
    for kind in ("forward", "backward", "fused"):
        n, ms = tim.get(kind, (0, 0.0))
        if n:
            per_iter = n / (steps * spec.iters * batches)
            b, f, fv, fm = step_work_split(spec, kind, vox / batches, per_iter, general)
            avg = ms / n / 1e3
            kinds[kind] = dict(launches=n, launches_per_iteration=per_iter, avg_ms=avg * 1e3, bytes=b, flops=f,
                               flops_valu=fv, flops_mfma=fm, gbs=b / avg / 1e9, tflops=f / avg / 1e12)
    return kinds


def lowrank_psfs(spec):
    """Non-separable rank-two PSFs for every view: the view's Gaussian plus 0.3 ×
    a Gaussian of twice its x width and half its z width, offset by 3 rows and
    −2 columns (a weaker side lobe), normalised; float32 [K][K]."""
    import numpy as np

    from synthetic import gaussian_psf

    out = []
    for sx, sz in spec.view_sigmas():
        side = np.roll(np.roll(gaussian_psf(spec.psf_k, 2.0 * sx, 0.5 * sz), 3, axis=0), -2, axis=1)
        p = gaussian_psf(spec.psf_k, sx, sz) + 0.3 * side
        out.append((p / p.sum()).astype(np.float32))
    return out


def host_cores():
    """Host threads this process may use (capped at 16, the machine's CPU share)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _oracle_job(job):
    """One worker's share of the CPU baseline: the oracle on its planes."""
    import numpy as np

    import oracle

    stacks, psfs, iters, update, normalize = job
    oracle.deconvolve(stacks, [np.asarray(p, dtype=np.float64) for p in psfs], iters, update=update,
                      normalize=normalize, method="fft")
    return True


def oracle_pool(jobs):
    """Run oracle jobs over worker processes (one job each, at most host_cores()
    at a time); returns (wall seconds of the timed map, workers used)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    workers = min(host_cores(), len(jobs))
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(_oracle_job, [jobs[0]] * workers))   # start and warm every worker
        t0 = time.perf_counter()
        list(ex.map(_oracle_job, jobs))
        return time.perf_counter() - t0, workers


def cpu_baseline(spec, vol, iters, normalize=False):
    """The float64 oracle on the host's cores: one plane per worker process, a
    seeded sample of the workload's planes, the oracle's FFT convolution mode
    (pinned to its direct sum)."""
    cores = host_cores()
    y0 = max(0, spec.n_planes // 2 - cores // 2)
    ys = list(range(y0, min(spec.n_planes, y0 + cores)))
    # about 10 iterations of a 512×512 plane per worker: larger planes time fewer iterations
    n_it = max(1, min(iters, (10 * 512 * 512) // (spec.n_z * spec.n_x)))
    jobs = [([s[:, y:y + 1, :].copy() for s in vol["stacks"]], vol["psfs"], n_it, spec.update, normalize)
            for y in ys]
    dt, workers = oracle_pool(jobs)
    vox_it = len(ys) * spec.n_z * spec.n_x * n_it
    which = f"all {iters}" if n_it == iters else f"{n_it} of {iters}"
    return {"value": vox_it / dt, "unit": "voxel-iterations/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(ys)} of {spec.n_planes} planes ({ys[0]}..{ys[-1]}), one per worker process, "
                      f"{which} iterations, {spec.n_views} views, FP64 FFT convolution, {dt:.1f} s"}


def mix_record(args, cpu=True):
    """Three uneven volumes: plain per-volume calls vs one batched launch (the
    tuned batch, which times the persistent work-queue form and the graph form
    and keeps the faster; both forms are also timed on their own).
    Returns a dict: batched and plain rates, their ratio, the largest relative
    difference between the two estimates, both forms' rates, the roofline of
    the mix's dominant kernel (from HIP-event timings of the plain calls) and
    the CPU baseline."""
    import numpy as np

    from synthetic import CONFIGS, make_volume

    specs = [CONFIGS["mix_a"], CONFIGS["mix_b"], CONFIGS["mix_c"]]
    vols = []
    workers = host_cores()
    for spec in specs:   # all inputs drawn before the GPU is touched
        log(f"generating {spec.name}: {spec.n_views} views, {spec.n_planes} planes of {spec.n_z}x{spec.n_x}, "
            f"K={spec.psf_k}")
        vols.append(make_volume(spec, truth=False, workers=workers))
    cpu_jobs = []
    for spec, vol in zip(specs, vols):   # one plane of each volume for the CPU baseline
        y = spec.n_planes // 2
        cpu_jobs.append(([np.ascontiguousarray(s[:, y:y + 1, :]) for s in vol["stacks"]], vol["psfs"], 1,
                         spec.update, False))
    import torch

    from paper_1503_07998_amd import api

    dev = torch.device("cuda:0")
    setups = []
    for spec, vol in zip(specs, vols):
        obs = [torch.from_numpy(s).to(dev) for s in vol["stacks"]]
        del vol["stacks"]
        d = api.Deconvolver(spec.n_views, spec.n_z, spec.n_x, 0)
        for v, p in enumerate(vol["psfs"]):
            d.set_psf(v, p)
        est = torch.empty((spec.n_planes, spec.n_z, spec.n_x), dtype=torch.float32, device=dev)
        runs = {}
        for timing in (False, True):
            runs[timing] = api.make_run(spec.n_planes, spec.iters, update=spec.update, boundary=spec.boundary,
                                        obs_dtype=spec.obs_dtype, layout="stack_zyx", tune=True, timing=timing)
        nb = api.mvd_workspace_bytes(d.ctx, runs[False])
        ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        for r in runs.values():
            r.workspace = (ws.data_ptr() + 255) // 256 * 256
            r.workspace_bytes = nb
        setups.append(dict(spec=spec, obs=obs, dec=d, est=est, runs=runs, ws=ws))
    vox_it = sum(sp.voxels * sp.iters for sp in specs)

    def plain_step(timing=False):   # tuned launch shapes too (first call), so only the single launch differs
        for st in setups:
            api.mvd_deconvolve_planes(st["dec"].ctx, st["obs"], st["est"], st["runs"][timing])

    log("mix: plain per-volume calls")
    for _ in range(args.warmup):
        plain_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain_step()
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    plain_out = [st["est"].cpu().numpy().copy() for st in setups]
    # launch durations of one plain step, per volume
    for st in setups:
        api.mvd_get_timing(st["dec"].ctx, reset=True)
    plain_step(timing=True)
    torch.cuda.synchronize()
    per_vol = []
    for st in setups:
        tim = api.mvd_get_timing(st["dec"].ctx, reset=True)
        kinds = launch_kinds(st["spec"], tim, 1, st["spec"].voxels)
        per_vol.append((st["spec"], kinds))

    entries = [(st["dec"].ctx, st["obs"], st["est"], st["runs"][False]) for st in setups]

    def time_batch(b):
        for _ in range(args.warmup):
            b.launch()
        b.wait()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.launch()
        b.wait()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        d = max(float(np.abs(st["est"].cpu().numpy() - ref).max() / np.abs(ref).max())
                for st, ref in zip(setups, plain_out))
        return ms, d

    log("mix: graph form (autotune + capture)")
    bg = api.Batch(entries, tune=True, graph=True)
    graph_ms, graph_diff = time_batch(bg)
    tuning = [bg.tuning(i) for i in range(len(setups))]
    bg.close()
    log("mix: persistent form")
    b = api.Batch(entries)
    pq_info = b.info()
    pq_ms, pq_diff = time_batch(b)
    b.close()
    log("mix: tuned batch (both forms timed, the faster kept)")
    b = api.Batch(entries, tune=True)
    info = b.info()
    form_times = b.form_times()
    batch_ms, diff = time_batch(b)
    b.close()
    # the dominant kernel of the mix: the (volume, pass) with the largest total launch time
    spec_d, kinds_d = max(per_vol, key=lambda sk: max(k["avg_ms"] * k["launches"] for k in sk[1].values()))
    roof = roofline(spec_d, kinds_d, variant=True)
    roof["kernel"] = f"{spec_d.name}: " + roof["kernel"]
    out = {
        "value": vox_it / (batch_ms / 1e3), "unit": "voxel-iterations/s", "ms_per_step": batch_ms,
        "plain_value": vox_it / (plain_ms / 1e3), "plain_ms_per_step": plain_ms,
        "batched_over_plain": plain_ms / batch_ms, "max_rel_diff_batched_vs_plain": diff,
        "batch_form": info, "batch_form_timed_ms": {"persistent": form_times[0], "graph": form_times[1]},
        "persistent_form_value": vox_it / (pq_ms / 1e3), "persistent_form_ms_per_step": pq_ms,
        "persistent_form_max_rel_diff": pq_diff, "persistent_form": pq_info,
        "graph_form_value": vox_it / (graph_ms / 1e3), "graph_form_ms_per_step": graph_ms,
        "graph_form_max_rel_diff": graph_diff,
        "workload": "batched mix: 200 planes 256x384 (2 views, 21x21), 300 planes 512x768 (3 views, 31x31), "
                    "150 planes 1000x1000 (4 views, 41x41), f32 Poisson observations, 10 sequential iterations, "
                    "zero boundary",
        "voxels": sum(sp.voxels for sp in specs), "tuning": tuning,
        "kernels": {sp.name: k for sp, k in per_vol},
        "roofline": roof,
    }
    for st in setups:
        st["dec"].close()
    del setups
    if cpu:
        log("mix: cpu baseline (oracle)")
        dt, w = oracle_pool(cpu_jobs)
        vi = sum(sp.n_z * sp.n_x for sp in specs)
        out["cpu_baseline"] = {
            "value": vi / dt, "unit": "voxel-iterations/s", "cores": w, "kind": "oracle",
            "sample": "the middle plane of each of the 3 volumes, one per worker process, 1 of 10 iterations, "
                      f"FP64 FFT convolution, {dt:.1f} s"}
    return out


def bench_mix(args):
    """--config mix: the batched-vs-plain record as its own JSON line."""
    rec = mix_record(args, cpu=not args.no_cpu_baseline)
    out = {
        "metric": "voxel-iterations/s", "value": rec["value"], "unit": "voxel-iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": rec["workload"], "voxels": rec["voxels"], "parallelism": "single GPU"},
    }
    out.update({k: v for k, v in rec.items() if k not in ("value", "unit", "ms_per_step", "workload", "voxels")})
    print(json.dumps(out), flush=True)


def bench_calibrate(args):
    """Kernels of known traffic.  The reslice of a float32 camera stack of
    1 GiB into float32 planes (every element read once and written once)
    calibrates the HBM byte counters; a plain copy of the same 1 GiB and a
    read-only sweep of it (16 bytes per lane, the library's calibration
    kernels) give the bandwidth a streaming kernel reaches on the device,
    the yardstick beside the 8 TB/s peak."""
    import ctypes

    import torch

    from paper_1503_07998_amd import _native as N
    from paper_1503_07998_amd import api

    Z, Y, X = 1024, 256, 1024    # 2^28 float32 values = 1 GiB
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(3)
    stack = torch.rand((Z, Y, X), generator=g, device=dev)
    planes = torch.empty((Y, Z, X), dtype=torch.float32, device=dev)
    nbytes = Z * Y * X * 4
    lib = N.lib()
    probe = lib.mvd_internal_stream_probe
    probe.restype = ctypes.c_int
    probe.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def run_probe(kind):
        st = probe(kind, stack.data_ptr(), planes.data_ptr(), nbytes, stream)
        if st != 0:
            raise N.MvdError(st, f"stream probe {kind} failed")

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    ctx = api.mvd_create(1, Z, X, 0)
    try:
        ms = timed(lambda: api.mvd_reslice(ctx, stack, Y, planes))
    finally:
        api.mvd_destroy(ctx)
    ms_copy = timed(lambda: run_probe(0))
    ms_read = timed(lambda: run_probe(1))
    rates = {"reslice_GBps": 2 * nbytes / (ms / 1e3) / 1e9, "copy_GBps": 2 * nbytes / (ms_copy / 1e3) / 1e9,
             "read_GBps": nbytes / (ms_read / 1e3) / 1e9}
    log("calibration: " + ", ".join(f"{k} {v:.0f}" for k, v in rates.items()))
    print(json.dumps({"metric": "GB/s", "value": rates["reslice_GBps"], "unit": "GB/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "reslice of a 1 GiB float32 stack (1024 slices of 256x1024) into "
                                             "planes: counter calibration, 1 GiB read + 1 GiB written per launch"},
                      "bytes_read": nbytes, "bytes_written": nbytes, "streaming": rates,
                      "ms_copy": ms_copy, "ms_read": ms_read}), flush=True)


def bench_stream(args, spec):
    """Observations in page-locked host memory, streamed to the device in
    batches of planes that overlap with the iterations of other batches.
    One step = the whole deconvolution, host stacks to device estimate."""
    import numpy as np

    from synthetic import make_volume

    Y, Z, X, V = spec.n_planes, spec.n_z, spec.n_x, spec.n_views
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    log(f"generating {spec.name}: {V} views, {Y} planes of {Z}x{X}, K={spec.psf_k} ({workers} workers)")
    t0 = time.perf_counter()
    vol = make_volume(spec, truth=False, workers=workers)
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    import torch

    from paper_1503_07998_amd import api

    host = []
    for v in range(V):
        t = torch.empty((Z, Y, X), dtype=torch.uint16, pin_memory=True)
        t.numpy()[...] = vol["stacks"][v]
        host.append(t)
    y_cpu = max(0, Y // 2 - host_cores() // 2)
    cpu_jobs = [([np.ascontiguousarray(s[:, y:y + 1, :]) for s in vol["stacks"]], vol["psfs"], 1, spec.update,
                 False) for y in range(y_cpu, min(Y, y_cpu + host_cores()))]
    del vol["stacks"]
    dev = torch.device("cuda:0")
    d = api.Deconvolver(V, Z, X, 0)
    for v, p in enumerate(vol["psfs"]):
        d.set_psf(v, p)
    est = torch.empty((Y, Z, X), dtype=torch.float32, device=dev)
    batch = args.batch
    nb = (Y + batch - 1) // batch

    def make(timing, ws_bytes, ptr):
        r = api.make_run(Y, spec.iters, update=spec.update, boundary=spec.boundary, obs_dtype=spec.obs_dtype,
                         timing=timing, tune=True)
        r.workspace, r.workspace_bytes = ptr, ws_bytes
        return r

    nbytes = api.mvd_stream_workspace_bytes(d.ctx, make(False, 0, None), batch, False)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    wptr = (ws.data_ptr() + 255) // 256 * 256
    runs = {t: make(t, nbytes, wptr) for t in (False, True)}
    stream = torch.cuda.current_stream()

    def timed(fn, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    log(f"streamed: batches of {batch} planes, warmup {args.warmup}")
    for _ in range(args.warmup):
        api.mvd_deconvolve_stream(d.ctx, host, est, runs[False], batch, stream)
    api.mvd_get_timing(d.ctx, reset=True)
    log(f"streamed: timing {args.steps} steps")
    ms_step = timed(lambda: api.mvd_deconvolve_stream(d.ctx, host, est, runs[True], batch, stream), args.steps)
    tim = api.mvd_get_timing(d.ctx, reset=True)
    ms_plain = timed(lambda: api.mvd_deconvolve_stream(d.ctx, host, est, runs[False], batch, stream), args.steps)
    vox_it = spec.voxels * spec.iters
    kinds = launch_kinds(spec, tim, args.steps, spec.voxels, nb)
    it_ms = sum(kinds[k]["avg_ms"] * kinds[k]["launches"] for k in kinds) / args.steps
    del ws

    # the same run with the estimate copied back to page-locked host memory
    log("streamed with host estimate")
    est_h = torch.empty((Y, Z, X), dtype=torch.float32, pin_memory=True)
    nbh = api.mvd_stream_workspace_bytes(d.ctx, runs[False], batch, True)
    wsh = torch.empty(nbh + 256, dtype=torch.uint8, device=dev)
    rh = make(False, nbh, (wsh.data_ptr() + 255) // 256 * 256)
    api.mvd_deconvolve_stream(d.ctx, host, est_h, rh, batch, stream)
    ms_host_out = timed(lambda: api.mvd_deconvolve_stream(d.ctx, host, est_h, rh, batch, stream), args.steps)
    same = bool(torch.equal(est_h, est.cpu()))
    del wsh, est_h

    # copies alone, and the device-resident run, for context
    log("host-to-device copy alone")
    obs = [torch.empty((Z, Y, X), dtype=torch.uint16, device=dev) for _ in range(V)]

    def copy_in():
        for o, h in zip(obs, host):
            o.copy_(h, non_blocking=True)

    copy_in()
    ms_copy = timed(copy_in, 2)
    log("device-resident run")
    rr = api.make_run(Y, spec.iters, update=spec.update, boundary=spec.boundary, obs_dtype=spec.obs_dtype,
                      tune=True)
    nr = api.mvd_workspace_bytes(d.ctx, rr)
    wsr = torch.empty(nr + 256, dtype=torch.uint8, device=dev)
    rr.workspace, rr.workspace_bytes = (wsr.data_ptr() + 255) // 256 * 256, nr
    api.mvd_deconvolve_planes(d.ctx, obs, est, rr, stream)
    ms_res = timed(lambda: api.mvd_deconvolve_planes(d.ctx, obs, est, rr, stream), max(1, args.steps // 2))
    del wsr, obs

    out = {
        "metric": "voxel-iterations/s",
        "value": vox_it / (ms_step / 1e3),
        "unit": "voxel-iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": (f"{spec.name}: {V} views (0/90/180/270 deg), {Y} planes of {Z}x{X}, "
                         f"{spec.psf_k}x{spec.psf_k} Gaussian PSFs (sx={spec.psf_sigma[0]}, sz={spec.psf_sigma[1]}), "
                         f"uint16 Poisson observations of blob nuclei in page-locked host memory streamed in "
                         f"batches of {batch} planes, {spec.iters} iterations, {spec.update}, "
                         f"{spec.boundary} boundary, estimate on the device"),
            "voxels": spec.voxels, "iterations": spec.iters, "views": V, "psf": spec.psf_k,
            "update": spec.update, "batch_planes": batch, "parallelism": "single GPU",
        },
        "ms_per_step_without_events": ms_plain,
        "iterations_only_value": vox_it / (it_ms / 1e3),
        "host_estimate_value": vox_it / (ms_host_out / 1e3),
        "host_estimate_equal": same,
        "h2d_copy_ms": ms_copy,
        "h2d_copy_gbs": V * spec.voxels * 2 / (ms_copy / 1e3) / 1e9,
        "device_resident_value": vox_it / (ms_res / 1e3),
        "device_resident_ms": ms_res,
        "kernels": kinds,
        "roofline": roofline(spec, kinds),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        dt, w = oracle_pool(cpu_jobs)
        out["cpu_baseline"] = {
            "value": len(cpu_jobs) * Z * X / dt, "unit": "voxel-iterations/s", "cores": w, "kind": "oracle",
            "sample": f"{len(cpu_jobs)} of {Y} planes, one per worker process, 1 of {spec.iters} iterations, "
                      f"{V} views, FP64 FFT convolution, {dt:.1f} s"}
    d.close()
    print(json.dumps(out), flush=True)


def bench_grad(args, spec):
    """Differentiation workload: ψ^T(σ, w) through the unrolled iterations with
    checkpoints, MSE to the ground truth, and the reverse sweep to ∂L/∂σ and
    ∂L/∂w (torch.autograd over the library's forward and adjoint).  One step =
    forward + loss + backward."""
    import numpy as np

    from synthetic import make_volume

    Y, Z, X, V, K = spec.n_planes, spec.n_z, spec.n_x, spec.n_views, spec.psf_k
    log(f"generating {spec.name}: {V} views, {Y} planes of {Z}x{X}, K={K}")
    vol = make_volume(spec)
    import torch

    from paper_1503_07998_amd import api
    from paper_1503_07998_amd.autograd import PlanewiseRL

    dev = torch.device("cuda:0")
    obs = [torch.from_numpy(s).to(dev) for s in vol["stacks"]]
    truth = torch.from_numpy(np.ascontiguousarray(np.transpose(vol["truth"], (1, 0, 2)))).to(dev)
    prob = PlanewiseRL(obs, K, spec.iters, update=spec.update, boundary=spec.boundary)
    sig0 = [[1.7, 6.6], [6.3, 1.6]][:V]
    w0 = [0.9, 0.8][:V]

    def step():
        sigma = torch.tensor(sig0, dtype=torch.float64, requires_grad=True)
        w = torch.tensor(w0, dtype=torch.float64, requires_grad=True)
        psi = prob(sigma, w)
        loss = ((psi - truth) ** 2).mean()
        loss.backward()
        return loss, sigma.grad, w.grad

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss, gs, gw = step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    prob.timing = True
    api.mvd_get_timing(prob.dec.ctx, reset=True)
    step()
    torch.cuda.synchronize()
    tim = api.mvd_get_timing(prob.dec.ctx, reset=True)
    prob.timing = False
    breakdown = {k: {"launches": n, "ms": ms} for k, (n, ms) in tim.items() if n}
    vox = spec.voxels
    n_corr, ms_corr = tim["correlation"]
    pairs = n_corr // 2                        # each tap gradient: one correlation + one finalize launch
    flops = 2.0 * K * K * vox                  # one K×K tap gradient over every voxel
    achieved = flops / (ms_corr / pairs / 1e3) / 1e12 if pairs else None
    valu_corr = "valu_corr=1" in os.environ.get("MVD_TUNE", "")
    corr_peak = ALU_PEAK if valu_corr else MFMA_F32_PEAK
    out = {
        "metric": "voxel-iterations/s",
        "value": vox * spec.iters / (ms_step / 1e3),
        "unit": "voxel-iterations/s (forward + reverse sweep)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": (f"{spec.name}: {V} views, {Y} planes of {Z}x{X}, {K}x{K} Gaussian PSFs, "
                         f"{spec.iters} {spec.update} iterations with checkpoints, MSE to the ground truth, "
                         f"gradients w.r.t. per-view (sx, sz) at {sig0} and weights {w0}"),
            "voxels": vox, "iterations": spec.iters, "views": V, "psf": K, "parallelism": "single GPU"},
        "loss": float(loss), "grad_sigma": gs.tolist(), "grad_weights": gw.tolist(),
        "launch_ms": breakdown,
        "roofline": {"bound": "alu" if valu_corr else "mfma", "achieved": achieved, "peak": corr_peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / (corr_peak / 1e12) if achieved else None,
                     "traffic": None,
                     "kernel": (f"tap-gradient correlation on the {'vector ALUs' if valu_corr else 'matrix cores'} "
                                f"({K}x{K} lags, 2 flop per lag and voxel)")},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle forward + reverse sweep on one plane)")
        from oracle import adjoint as OA

        y = Y // 2
        phis = [np.ascontiguousarray(np.transpose(s_[:, y:y + 1, :], (1, 0, 2))).astype(np.float64)
                for s_ in vol["stacks"]]
        tr = np.ascontiguousarray(np.transpose(vol["truth"][:, y:y + 1, :], (1, 0, 2))).astype(np.float64)
        t0 = time.perf_counter()
        OA.sigma_gradients(phis, sig0, w0, spec.iters, tr, K, spec.update, spec.boundary)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": Z * X * spec.iters / dt, "unit": "voxel-iterations/s (forward + reverse sweep)", "cores": 1,
            "kind": "oracle",
            "sample": f"1 of {Y} planes (plane {y}), all {spec.iters} iterations forward and reverse, {V} views, "
                      f"direct FP64 convolution, {dt:.1f} s"}
    prob.dec.close()
    print(json.dumps(out), flush=True)


def write_stack(path, t, chunk=64):
    """Writes a device tensor [Z][Y][X] to a raw file, chunk slices at a time,
    then flushes it and drops it from the page cache (so it is read from disk)."""
    fd = os.open(path, os.O_WRONLY | os.O_CREAT | os.O_TRUNC, 0o644)
    try:
        for z0 in range(0, t.shape[0], chunk):
            buf = t[z0:z0 + chunk].cpu().numpy().tobytes()
            view = memoryview(buf)
            while view:
                n = os.write(fd, view)
                view = view[n:]
        os.fsync(fd)
        os.posix_fadvise(fd, 0, 0, os.POSIX_FADV_DONTNEED)
    finally:
        os.close(fd)


def bench_vol2048(args, spec):
    """The whole 2048³ volume (2 views, 10 iterations): device-resident, then,
    with --disk DIR, the same run disk to disk (stacks read from raw files in
    DIR, ψ^T written to a raw file there, page cache dropped behind every read
    and write).  The observations are a slab of --distinct rendered planes
    repeated along the plane axis on the device (planes are deconvolved
    independently, so the per-plane work is that of a fully rendered volume)."""
    import shutil
    import tempfile

    import numpy as np
    import torch

    from paper_1503_07998_amd import api
    from synthetic import make_volume

    Y, Z, X = spec.n_planes, spec.n_z, spec.n_x
    nd = args.distinct
    if nd < 1 or Y % nd:
        raise SystemExit(f"--distinct must divide {Y}")
    log(f"generating a {nd}-plane slab of {spec.name}")
    t0 = time.perf_counter()
    vol = make_volume(spec, planes=nd, truth=False, workers=host_cores())
    log(f"generated in {time.perf_counter() - t0:.1f} s; repeating it {Y // nd}x along the plane axis")
    dev = torch.device("cuda:0")
    obs = [torch.from_numpy(s).to(dev).repeat(1, Y // nd, 1) for s in vol["stacks"]]
    d = api.Deconvolver(spec.n_views, Z, X, 0)
    for v, p in enumerate(vol["psfs"]):
        d.set_psf(v, p)
    est = torch.empty((Y, Z, X), dtype=torch.float32, device=dev)

    def make(timing):
        return api.make_run(Y, spec.iters, update=spec.update, boundary=spec.boundary, obs_dtype="u16",
                            layout="stack_zyx", timing=timing, tune=True)

    nbytes = api.mvd_workspace_bytes(d.ctx, make(False))
    log(f"device memory: stacks {2 * sum(o.numel() for o in obs) / 1e9:.1f} GB, estimate "
        f"{est.numel() * 4 / 1e9:.1f} GB, workspace {nbytes / 1e9:.1f} GB")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    wptr = (ws.data_ptr() + 255) // 256 * 256
    runs = {}
    for timing in (False, True):
        r = make(timing)
        r.workspace = wptr
        r.workspace_bytes = nbytes
        runs[timing] = r
    stream = torch.cuda.current_stream()
    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        api.mvd_deconvolve_planes(d.ctx, obs, est, runs[False], stream)
    torch.cuda.synchronize()
    api.mvd_get_timing(d.ctx, reset=True)
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        api.mvd_deconvolve_planes(d.ctx, obs, est, runs[True], stream)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    tim = api.mvd_get_timing(d.ctx, reset=True)
    vox_it = spec.voxels * spec.iters
    kinds = launch_kinds(spec, tim, args.steps, Y * Z * X)
    out = {
        "metric": "voxel-iterations/s",
        "value": vox_it / (ms_step / 1e3),
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{spec.name}: {spec.n_views} views, {Y} planes of {Z}x{X}, {spec.psf_k}x{spec.psf_k} "
                         f"Gaussian PSFs (sx={spec.psf_sigma[0]}, sz={spec.psf_sigma[1]}, view 1 rotated 90 deg), "
                         f"u16 Poisson observations of blob nuclei ({nd} rendered planes repeated along the plane "
                         f"axis), {spec.iters} iterations, {spec.update}, {spec.boundary} boundary, "
                         "device-resident"),
            "voxels": spec.voxels, "iterations": spec.iters, "views": spec.n_views,
            "psf": spec.psf_k, "update": spec.update, "parallelism": "single GPU",
        },
        "kernels": kinds,
        "roofline": roofline(spec, kinds),
        "paper_context": PAPER_CONTEXT.get(spec.name),
    }
    del ws, runs
    torch.cuda.empty_cache()
    if args.disk:
        ddir = tempfile.mkdtemp(dir=args.disk, prefix="mvd_vol2048.")
        try:
            paths = [os.path.join(ddir, f"view{v}.u16") for v in range(spec.n_views)]
            log(f"writing the stacks to {ddir}")
            t0 = time.perf_counter()
            for p, o in zip(paths, obs):
                write_stack(p, o)
            log(f"wrote {2 * sum(o.numel() for o in obs) / 1e9:.1f} GB in {time.perf_counter() - t0:.1f} s")
            est_path = os.path.join(ddir, "estimate.f32")
            run = api.make_run(Y, spec.iters, update=spec.update, boundary=spec.boundary, obs_dtype="u16",
                               layout="stack_zyx", tune=True)
            nb = api.mvd_stream_workspace_bytes(d.ctx, run, args.batch, True)
            ws2 = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
            run.workspace = (ws2.data_ptr() + 255) // 256 * 256
            run.workspace_bytes = nb
            fds = [os.open(p, os.O_RDONLY) for p in paths]
            efd = os.open(est_path, os.O_RDWR | os.O_CREAT | os.O_TRUNC, 0o644)
            try:
                log(f"disk-to-disk run: batches of {args.batch} planes, {args.io_threads} I/O threads")
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = api.mvd_deconvolve_files(d.ctx, fds, efd, run, args.batch, io_threads=args.io_threads,
                                              sync=True, drop_cache=True, stream=stream)
                wall = time.perf_counter() - t0
                # a few planes of the file against the device-resident result
                diff = 0.0
                for y in (0, Y // 2, Y - 1):
                    got = np.fromfile(est_path, dtype=np.float32, count=Z * X, offset=y * Z * X * 4)
                    ref = est[y].cpu().numpy().ravel()
                    diff = max(diff, float(np.abs(got - ref).max() / np.abs(ref).max()))
            finally:
                for fd in fds + [efd]:
                    os.close(fd)
            out["disk"] = {
                "value": vox_it / wall, "unit": "voxel-iterations/s", "seconds": wall,
                "workload": (f"the same run disk to disk: stacks read from raw uint16 files, estimate written as "
                             f"raw float32 planes, batches of {args.batch} planes, 3 page-locked batches per "
                             f"direction, {args.io_threads} I/O threads, page cache dropped behind every read and "
                             "write, estimate file fdatasync'ed"),
                "read_s": st["read_s"], "write_s": st["write_s"], "wait_for_reads_s": st["wait_s"],
                "bytes_read": st["bytes_read"], "bytes_written": st["bytes_written"],
                "read_gbs": st["bytes_read"] / st["read_s"] / 1e9 if st["read_s"] else None,
                "write_gbs": st["bytes_written"] / st["write_s"] / 1e9 if st["write_s"] else None,
                "max_rel_diff_vs_device_resident": diff,
                "paper_context": PAPER_CONTEXT.get(spec.name),
            }
            log(f"disk run: {wall:.1f} s; read {st['read_s']:.1f} s, write {st['write_s']:.1f} s")
        finally:
            shutil.rmtree(ddir, ignore_errors=True)
    d.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="vol512")
    ap.add_argument("--update", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=64, help="planes per streamed batch (vol1024x4)")
    ap.add_argument("--force-2d", action="store_true",
                    help="run the general KxK passes even for rank-one PSFs (default workload)")
    ap.add_argument("--normalize", action="store_true",
                    help="EM-normalised back-projection (divide by X (*) 1; default workload)")
    ap.add_argument("--pixel-weights", action="store_true",
                    help="per-pixel view weights (seeded uniform [0.5, 1] planes; default workload)")
    ap.add_argument("--no-mix", action="store_true",
                    help="leave out the batched-vs-plain mix record of the default run")
    ap.add_argument("--disk", default=None, metavar="DIR",
                    help="vol2048: also run disk to disk with the files in DIR (needs ~70 GB free)")
    ap.add_argument("--distinct", type=int, default=32,
                    help="vol2048: rendered planes repeated along the plane axis")
    ap.add_argument("--io-threads", type=int, default=8, help="vol2048 --disk: threads per read or write")
    ap.add_argument("--psf-k", type=int, default=0, help="PSF side (default workload; 0: the workload's)")
    ap.add_argument("--no-tune", action="store_true",
                    help="untuned launch shapes (MVD_TUNE overrides apply; default workload)")
    ap.add_argument("--psf", default="gauss", choices=["gauss", "lowrank"],
                    help="lowrank: deconvolve with non-separable rank-two PSFs (a main lobe and a weaker, "
                         "wider offset lobe per view; default workload)")
    args = ap.parse_args()
    global WEIGHT_PLANES, PSF_TERMS
    WEIGHT_PLANES = args.pixel_weights
    PSF_TERMS = 2 if args.psf == "lowrank" else 1
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU (no multi-GPU path is built); "
                                   "--gpus must be 1", "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    if args.config == "mix":
        bench_mix(args)
        return
    if args.config == "calibrate":
        bench_calibrate(args)
        return

    from synthetic import CONFIGS, make_volume

    spec = CONFIGS[args.config]
    if args.update:
        spec.update = args.update
    if args.psf_k:
        spec.psf_k = args.psf_k
    if spec.name == "vol1024x4":
        bench_stream(args, spec)
        return
    if spec.name == "grad256":
        bench_grad(args, spec)
        return
    if spec.name == "vol2048":
        bench_vol2048(args, spec)
        return
    log(f"generating {spec.name}: {spec.n_views} views, {spec.n_planes} planes of {spec.n_z}x{spec.n_x}")
    t0 = time.perf_counter()
    vol = make_volume(spec, truth=False, workers=max(1, min(16, len(os.sched_getaffinity(0)))))
    log(f"generated in {time.perf_counter() - t0:.1f} s")

    import numpy as np
    import torch

    from paper_1503_07998_amd import api

    dev = torch.device("cuda:0")
    obs = [torch.from_numpy(s).to(dev) for s in vol["stacks"]]
    Y, Z, X = spec.n_planes, spec.n_z, spec.n_x
    layout = "stack_zyx"
    d = api.Deconvolver(spec.n_views, Z, X, 0)
    psfs = vol["psfs"] if args.psf == "gauss" else lowrank_psfs(spec)
    for v, p in enumerate(psfs):
        d.set_psf(v, p)
    if args.psf == "lowrank":
        forms = [api.mvd_psf_info(d.ctx, v) for v in range(spec.n_views)]
        log(f"PSF terms per view (PSF, back-projector): {forms}")
    est = torch.empty((Y, Z, X), dtype=torch.float32, device=dev)
    obs_dtype = "u16" if spec.obs_dtype == "u16" else "f32"

    wplanes = None
    if args.pixel_weights:
        g = torch.Generator(device=dev).manual_seed(7)
        wplanes = [0.5 + 0.5 * torch.rand((Y, Z, X), generator=g, device=dev) for _ in range(spec.n_views)]

    def make(timing):
        return api.make_run(Y, spec.iters, update=spec.update, boundary=spec.boundary,
                            obs_dtype=obs_dtype, layout=layout, timing=timing,
                            tune=not (args.force_2d or args.no_tune),
                            force_2d=args.force_2d, normalize=args.normalize, weight_planes=wplanes)

    run = make(False)
    nbytes = api.mvd_workspace_bytes(d.ctx, run)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    wptr = (ws.data_ptr() + 255) // 256 * 256
    runs = {}
    for timing in (False, True):
        r = make(timing)
        r.workspace = wptr
        r.workspace_bytes = nbytes
        runs[timing] = r
    stream = torch.cuda.current_stream()

    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        api.mvd_deconvolve_planes(d.ctx, obs, est, runs[False], stream)
    torch.cuda.synchronize()

    # timed region: K whole steps, launch durations recorded with HIP events
    api.mvd_get_timing(d.ctx, reset=True)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        api.mvd_deconvolve_planes(d.ctx, obs, est, runs[True], stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tim = api.mvd_get_timing(d.ctx, reset=True)
    ms_step = wall * 1e3 / args.steps
    vox_it = spec.voxels * spec.iters
    value = vox_it / (ms_step / 1e3)

    # untimed-event check of the same step (events themselves cost a little)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        api.mvd_deconvolve_planes(d.ctx, obs, est, runs[False], stream)
    torch.cuda.synchronize()
    ms_plain = (time.perf_counter() - t1) * 1e3 / args.steps

    kinds = launch_kinds(spec, tim, args.steps, Y * Z * X, general=args.force_2d)
    roof = roofline(spec, kinds, general=args.force_2d,
                    variant=args.normalize or args.pixel_weights or args.psf != "gauss")
    if roof.get("unit") == "GB/s":
        # context beside the peak: what a plain copy kernel streams on this device, measured now
        cr = copy_rate_gbs()
        roof["achievable"] = {"copy_GBps": cr, "frac_of_copy": roof["achieved"] / cr,
                              "source": "the library's copy kernel over 1 GiB (1 GiB read + 1 GiB written), "
                                        "HIP events, same process after the timed region"}

    it_ms = sum(kinds[k]["avg_ms"] * kinds[k]["launches"] for k in kinds) / args.steps
    out = {
        "metric": "voxel-iterations/s",
        "value": value,
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{spec.name}: {spec.n_views} views, {Y} planes of {Z}x{X}, "
                         f"{spec.psf_k}x{spec.psf_k} Gaussian PSFs (sx={spec.psf_sigma[0]}, "
                         f"sz={spec.psf_sigma[1]}, view 1 rotated 90 deg), {spec.obs_dtype} Poisson "
                         f"observations of blob nuclei, {spec.iters} iterations, {spec.update}, "
                         f"{spec.boundary} boundary"
                         + (", deconvolved with non-separable rank-two PSFs (main lobe + 0.3 x wider offset "
                            "lobe)" if args.psf == "lowrank" else "")
                         + (", general KxK passes forced (no rank-one split)" if args.force_2d else "")
                         + (", EM-normalised back-projection" if args.normalize else "")
                         + (", per-pixel view weights" if args.pixel_weights else "")),
            "voxels": spec.voxels, "iterations": spec.iters, "views": spec.n_views,
            "psf": spec.psf_k, "update": spec.update, "parallelism": "single GPU",
        },
        "ms_per_step_without_events": ms_plain,
        "iterations_only_value": vox_it / (it_ms / 1e3),
        "kernels": kinds,
        "roofline": roof,
        "paper_context": PAPER_CONTEXT.get(spec.name),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(spec, dict(vol, psfs=psfs), spec.iters, normalize=args.normalize)
    d.close()
    del obs, est, ws, runs, wplanes
    torch.cuda.empty_cache()
    plain = not (args.force_2d or args.normalize or args.pixel_weights or args.update or args.psf != "gauss"
                 or args.psf_k or args.no_tune)
    if spec.name == "vol512" and plain and not args.no_mix:
        out["mix"] = mix_record(args, cpu=not args.no_cpu_baseline)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
