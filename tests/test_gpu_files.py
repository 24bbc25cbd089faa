"""The disk-to-disk form (mvd_deconvolve_files) and the whole 2048³ volume.

The disk-to-disk form reads camera-ordered stacks from files and writes ψ^T to
a file, batch by batch (Supplementary Note 2 §3, Algorithm 1).  Planes are
independent, so its output must equal the device-resident whole-volume run
bitwise, for ragged batch counts, header offsets in the files, both
observation types and every host-slot count.

The 2048³ case (2 views, 2048 planes of 2048×2048, 31×31 PSFs, 10 iterations,
the largest size of Supplementary Table 1) runs device-resident in the launch
configuration the benchmark times.  Three planes hold rendered blob data and
are checked against the oracle; every other plane holds the same filler data
(background plus a column pattern) and is checked against the oracle's result
for that plane, so every plane of the volume is compared with the oracle.  A
second, sequential run checks every plane's flux: after the last sequential
sub-step a plane's total equals the last view's observed total (the adjoint
identity of the back-projector X = P^*).
"""
import concurrent.futures as cf
import multiprocessing as mp
import os

import numpy as np
import pytest

import oracle
from synthetic import CONFIGS, VolumeSpec, make_volume, render_planes

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _torch():
    import torch
    return torch


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _ctx(spec, psfs):
    from paper_1503_07998_amd import api

    d = api.Deconvolver(spec.n_views, spec.n_z, spec.n_x, 0)
    for v, p in enumerate(psfs):
        d.set_psf(v, p)
    return d


def _workspace(nbytes):
    torch = _torch()
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda:0")
    return ws, (ws.data_ptr() + 255) // 256 * 256


def _plain(d, spec, stacks, weight_planes=None):
    from paper_1503_07998_amd import api

    torch = _torch()
    Z, Y, X = stacks[0].shape
    obs = [torch.from_numpy(s).to("cuda:0") for s in stacks]
    est = torch.empty((Y, Z, X), dtype=torch.float32, device="cuda:0")
    run = api.make_run(Y, spec.iters, update=spec.update, obs_dtype=spec.obs_dtype, weight_planes=weight_planes)
    nb = api.mvd_workspace_bytes(d.ctx, run)
    ws, run.workspace = _workspace(nb)
    run.workspace_bytes = nb
    api.mvd_deconvolve_planes(d.ctx, obs, est, run)
    torch.cuda.synchronize()
    return est.cpu().numpy()


def _files(d, spec, stacks, tmp_path, batch, offsets, est_offset=0, weight_planes=None, **kw):
    """Writes the stacks to files (after `offsets[v]` bytes of 0xEE), runs the
    disk-to-disk form and returns (ψ^T read back, the estimate file's bytes
    before est_offset, the call's statistics)."""
    from paper_1503_07998_amd import api

    Z, Y, X = stacks[0].shape
    paths = []
    for v, s in enumerate(stacks):
        p = tmp_path / f"view{v}.raw"
        p.write_bytes(b"\xee" * offsets[v] + s.tobytes())
        paths.append(p)
    ep = tmp_path / "est.raw"
    ep.write_bytes(b"\x5a" * est_offset)
    run = api.make_run(Y, spec.iters, update=spec.update, obs_dtype=spec.obs_dtype, weight_planes=weight_planes)
    nb = api.mvd_stream_workspace_bytes(d.ctx, run, batch, True)
    ws, run.workspace = _workspace(nb)
    run.workspace_bytes = nb
    fds = [os.open(str(p), os.O_RDONLY) for p in paths]
    efd = os.open(str(ep), os.O_RDWR)
    try:
        st = api.mvd_deconvolve_files(d.ctx, fds, efd, run, batch, obs_offsets=offsets, est_offset=est_offset, **kw)
    finally:
        for fd in fds + [efd]:
            os.close(fd)
    raw = ep.read_bytes()
    assert len(raw) == est_offset + Y * Z * X * 4
    est = np.frombuffer(raw[est_offset:], dtype=np.float32).reshape(Y, Z, X)
    return est, raw[:est_offset], st


@pytest.mark.parametrize("slots", [0, 2, 5])
def test_files_equal_device_run(tmp_path, slots):
    """37 planes in batches of 8 (a short last batch), uint16 stacks after
    headers of different sizes, estimate after a header that must survive."""
    _say(f"disk-to-disk u16, 37 planes of 48x40, batch 8, host slots {slots}")
    spec = VolumeSpec("files_u16", 37, 48, 40, 7, (1.2, 2.5), (0, 90), 40, "u16", 4, "simultaneous", seed=91)
    vol = make_volume(spec, truth=False)
    d = _ctx(spec, vol["psfs"])
    ref = _plain(d, spec, vol["stacks"])
    got, head, st = _files(d, spec, vol["stacks"], tmp_path, 8, [4096, 100], est_offset=512, host_slots=slots,
                           io_threads=3)
    d.close()
    np.testing.assert_array_equal(got, ref)
    assert head == b"\x5a" * 512
    assert st["bytes_read"] == 2 * 48 * 37 * 40 * 2
    assert st["bytes_written"] == 37 * 48 * 40 * 4
    assert st["wall_s"] > 0 and st["read_s"] >= 0 and st["write_s"] >= 0
    ora = oracle.deconvolve([s[:, 20:22, :] for s in vol["stacks"]], [p.astype(np.float64) for p in vol["psfs"]],
                            spec.iters, update=spec.update)
    err = np.abs(got[20:22] - ora).max() / np.abs(ora).max()
    assert err <= TOL, err


def test_files_one_batch_f32_sequential(tmp_path):
    """A batch larger than the volume (one contiguous read per view), float32
    stacks, sequential updates, 3 views, with flushing and cache dropping."""
    _say("disk-to-disk f32, 3 views, one batch, sync + drop cache")
    spec = VolumeSpec("files_f32", 13, 33, 72, 9, (1.2, 2.5), (0, 90, 180), 20, "f32", 3, "sequential", seed=92)
    vol = make_volume(spec, truth=False)
    d = _ctx(spec, vol["psfs"])
    ref = _plain(d, spec, vol["stacks"])
    got, _, st = _files(d, spec, vol["stacks"], tmp_path, 64, [0, 8, 12], sync=True, drop_cache=True,
                        io_threads=1)
    # a second call on the same context reuses its page-locked batches
    got2, _, _ = _files(d, spec, vol["stacks"], tmp_path, 5, [0, 8, 12], io_threads=2)
    d.close()
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(got2, ref)
    assert st["bytes_read"] == 3 * 33 * 13 * 72 * 4


def test_files_with_weight_planes_equal_device_run(tmp_path):
    """Device-resident weight planes in the disk-to-disk form: bitwise the
    device-resident weighted run, 29 planes in batches of 6."""
    torch = _torch()
    _say("disk-to-disk u16 with weight planes, 29 planes of 40x48, batch 6")
    spec = VolumeSpec("files_w", 29, 40, 48, 9, (1.2, 2.5), (0, 90), 40, "u16", 3, "simultaneous", seed=94)
    vol = make_volume(spec, truth=False)
    d = _ctx(spec, vol["psfs"])
    rng = np.random.default_rng(95)
    planes = [torch.from_numpy(rng.uniform(0.2, 1.0, (29, 40, 48)).astype(np.float32)).to("cuda:0")
              for _ in range(2)]
    ref = _plain(d, spec, vol["stacks"], weight_planes=planes)
    got, _, _ = _files(d, spec, vol["stacks"], tmp_path, 6, [0, 0], weight_planes=planes)
    d.close()
    np.testing.assert_array_equal(got, ref)


def test_files_rejects_short_file(tmp_path):
    """A stack file that ends before its stack does is refused before any
    device work, and the estimate file stays untouched."""
    from paper_1503_07998_amd import _native as N

    _say("disk-to-disk: short file refused")
    spec = VolumeSpec("files_short", 6, 16, 16, 5, (1.2, 2.5), (0, 90), 4, "u16", 2, "simultaneous", seed=93)
    vol = make_volume(spec, truth=False)
    d = _ctx(spec, vol["psfs"])
    with pytest.raises(N.MvdError) as e:
        _files(d, spec, [vol["stacks"][0], vol["stacks"][1][:-1]], tmp_path, 2, [0, 0])
    assert e.value.status == N.MVD_ERR_ARG and "holds no" in str(e.value)
    assert (tmp_path / "est.raw").read_bytes() == b""
    d.close()


def _filler(Z, X):
    a = np.full((Z, X), 100, dtype=np.uint16)
    a[:, ::7] = 103
    return a


def test_vol2048_whole_volume():
    """2 views, 2048 planes of 2048×2048, 31×31, uint16, 10 iterations, whole
    volume on the device, tuned launch shapes (the benchmark's configuration)."""
    from paper_1503_07998_amd import api

    torch = _torch()
    spec = CONFIGS["vol2048"]
    Z, Y, X = spec.n_z, spec.n_planes, spec.n_x
    sample = [0, 1023, 2047]
    psfs = spec.psfs()
    p64 = [p.astype(np.float64) for p in psfs]
    torch.cuda.empty_cache()
    _say("vol2048: render sampled planes")
    real = render_planes(spec, sample)
    fill = _filler(Z, X)
    jobs = [[r[:, i:i + 1, :] for r in real] for i in range(len(sample))] + [[fill[:, None, :]] * 2]
    _say("vol2048: oracle on 3 sampled planes and the filler plane (4 processes)")
    pool = cf.ProcessPoolExecutor(len(jobs), mp_context=mp.get_context("spawn"))
    futs = [pool.submit(oracle.deconvolve, j, p64, spec.iters, update="simultaneous", method="fft") for j in jobs]
    try:
        obs = []
        for v in range(2):
            t = torch.from_numpy(fill).to("cuda:0")[:, None, :].repeat(1, Y, 1)
            for i, y in enumerate(sample):
                t[:, y, :] = torch.from_numpy(real[v][:, i, :]).to("cuda:0")
            obs.append(t)
        est = torch.empty((Y, Z, X), dtype=torch.float32, device="cuda:0")
        d = _ctx(spec, psfs)
        run = api.make_run(Y, spec.iters, update="simultaneous", obs_dtype="u16", tune=True)
        seq = api.make_run(Y, spec.iters, update="sequential", obs_dtype="u16")
        nb = max(api.mvd_workspace_bytes(d.ctx, run), api.mvd_workspace_bytes(d.ctx, seq))
        ws, base = _workspace(nb)
        for r in (run, seq):
            r.workspace = base
            r.workspace_bytes = nb
        _say(f"vol2048: simultaneous run (workspace {nb / 1e9:.0f} GB)")
        api.mvd_deconvolve_planes(d.ctx, obs, est, run)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(est).all()) and float(est.min()) >= 0.0
        refs = [f.result() for f in futs]
        _say("vol2048: every plane against the oracle")
        for i, y in enumerate(sample):
            got = est[y].cpu().numpy()
            err = np.abs(got - refs[i][0]).max() / np.abs(refs[i][0]).max()
            assert err <= TOL, f"plane {y}: max|d|/max = {err:.3e}"
        rf = torch.from_numpy(refs[-1][0].astype(np.float32)).to("cuda:0")
        worst = 0.0
        for y0 in range(0, Y, 128):
            e = ((est[y0:y0 + 128] - rf).abs().amax(dim=(1, 2)) / rf.abs().max()).cpu().numpy()
            for j, val in enumerate(e):
                if y0 + j not in sample:
                    worst = max(worst, float(val))
        assert worst <= TOL, f"filler planes: max|d|/max = {worst:.3e}"
        _say("vol2048: sequential run, flux of every plane")
        api.mvd_deconvolve_planes(d.ctx, obs, est, seq)
        torch.cuda.synchronize()
        obs_sum = torch.zeros(Y, dtype=torch.float64, device="cuda:0")
        for z0 in range(0, Z, 128):
            obs_sum += obs[-1][z0:z0 + 128].to(torch.float64).sum(dim=(0, 2))
        est_sum = torch.cat([est[y0:y0 + 128].to(torch.float64).sum(dim=(1, 2)) for y0 in range(0, Y, 128)])
        rel = ((est_sum - obs_sum).abs() / obs_sum).cpu().numpy()
        assert rel.max() <= 1e-5, f"flux identity off by {rel.max():.3e} at plane {rel.argmax()}"
        d.close()
        del obs, est, ws
    finally:
        pool.shutdown(wait=True, cancel_futures=True)
        torch.cuda.empty_cache()
