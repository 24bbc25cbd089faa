"""Streamed runs (mvd_deconvolve_stream) against the device-resident path and
the oracle.

Planes are independent, so a run over batches of planes copied from host
memory must equal the whole-volume run bitwise, whatever the batch size, the
estimate's placement (device or page-locked host) or the initial estimate.
At the 4-view 1024-plane size the check is on sampled planes against the
oracle plus a property of every plane: after the last sequential sub-step
(view V−1, weight 1) a plane's total equals that view's observed total
(adjoint identity of the back-projector X = P^*).
"""
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


def _pinned(a):
    torch = _torch()
    t = torch.empty(a.shape, dtype={np.uint16: torch.uint16, np.float32: torch.float32}[a.dtype.type],
                    pin_memory=True)
    t.numpy()[...] = a
    return t


def _plain(d, spec, stacks, init=None, weight_planes=None):
    """Whole-volume device-resident run."""
    from paper_1503_07998_amd import api

    torch = _torch()
    Z, Y, X = stacks[0].shape
    obs = [torch.from_numpy(s).to("cuda:0") for s in stacks]
    est = torch.empty((Y, Z, X), dtype=torch.float32, device="cuda:0")
    kw = {}
    if init is not None:
        est.copy_(torch.from_numpy(init))
        kw["init"] = "given"
    run = api.make_run(Y, spec.iters, update=spec.update, obs_dtype=spec.obs_dtype, weight_planes=weight_planes,
                       **kw)
    ws, run.workspace = _workspace(api.mvd_workspace_bytes(d.ctx, run))
    run.workspace_bytes = api.mvd_workspace_bytes(d.ctx, run)
    api.mvd_deconvolve_planes(d.ctx, obs, est, run)
    torch.cuda.synchronize()
    return est.cpu().numpy()


def _streamed(d, spec, host_obs, batch, est_host, init=None, Y=None, tune=False, weight_planes=None):
    from paper_1503_07998_amd import api

    torch = _torch()
    Z, Yh, X = host_obs[0].shape
    Y = Yh if Y is None else Y
    if est_host:
        est = torch.empty((Y, Z, X), dtype=torch.float32, pin_memory=True)
    else:
        est = torch.empty((Y, Z, X), dtype=torch.float32, device="cuda:0")
    kw = {}
    if init is not None:
        est.copy_(torch.from_numpy(init))
        kw["init"] = "given"
    else:
        est.fill_(-7.0)
    run = api.make_run(Y, spec.iters, update=spec.update, obs_dtype=spec.obs_dtype, tune=tune,
                       weight_planes=weight_planes, **kw)
    nb = api.mvd_stream_workspace_bytes(d.ctx, run, batch, est_host)
    ws, run.workspace = _workspace(nb)
    run.workspace_bytes = nb
    api.mvd_deconvolve_stream(d.ctx, host_obs, est, run, batch)
    torch.cuda.current_stream().synchronize()
    out = est.cpu().numpy().copy() if not est_host else est.numpy().copy()
    return out


SMALL = VolumeSpec("stream_small", 37, 48, 40, 9, (1.5, 3.0), (0, 90, 180, 270), 60, "u16", 4,
                   "sequential", seed=77)


@pytest.fixture(scope="module")
def small_case():
    vol = make_volume(SMALL, truth=False)
    d = _ctx(SMALL, vol["psfs"])
    plain = _plain(d, SMALL, vol["stacks"])
    host = [_pinned(s) for s in vol["stacks"]]
    yield dict(vol=vol, d=d, plain=plain, host=host)
    d.close()


@pytest.mark.parametrize("batch", [5, 37])
def test_streamed_weight_planes_equal_plain(small_case, batch):
    """Per-pixel weight planes stay on the device and each batch reads its
    own planes: bitwise the device-resident weighted run (and not the
    unweighted one); host weight planes are refused."""
    from paper_1503_07998_amd import _native as N

    torch = _torch()
    _say(f"streamed 37 planes with weight planes, batch={batch}")
    rng = np.random.default_rng(5)
    Z, Y, X = small_case["vol"]["stacks"][0].shape
    planes = [torch.from_numpy(rng.uniform(0.2, 1.0, (Y, Z, X)).astype(np.float32)).to("cuda:0")
              for _ in range(SMALL.n_views)]
    ref = _plain(small_case["d"], SMALL, small_case["vol"]["stacks"], weight_planes=planes)
    got = _streamed(small_case["d"], SMALL, small_case["host"], batch, True, weight_planes=planes)
    np.testing.assert_array_equal(got, ref)
    assert not np.array_equal(got, small_case["plain"])
    host_planes = [_pinned(p.cpu().numpy()) for p in planes]
    with pytest.raises(N.MvdError) as e:
        _streamed(small_case["d"], SMALL, small_case["host"], batch, True, weight_planes=host_planes)
    assert e.value.status == N.MVD_ERR_ARG and "device memory" in str(e.value)


@pytest.mark.parametrize("batch", [1, 8, 16, 37, 64])
@pytest.mark.parametrize("est_host", [False, True], ids=["est_dev", "est_host"])
def test_streamed_equals_plain(small_case, batch, est_host):
    _say(f"streamed 37 planes batch={batch} est_host={est_host}")
    got = _streamed(small_case["d"], SMALL, small_case["host"], batch, est_host)
    np.testing.assert_array_equal(got, small_case["plain"])


@pytest.mark.parametrize("est_host", [False, True], ids=["est_dev", "est_host"])
def test_streamed_tuned(small_case, est_host):
    """Launch shapes timed on the first batch: equal to the plain run up to
    float32 rounding, twice in a row (the second call uses the cached choice)."""
    _say(f"streamed with tuning est_host={est_host}")
    for rep in range(2):
        got = _streamed(small_case["d"], SMALL, small_case["host"], 8, est_host, tune=True)
        err = np.abs(got - small_case["plain"]).max() / np.abs(small_case["plain"]).max()
        assert err <= 1e-6, f"tuned streamed vs plain: {err:.3e} (call {rep})"


def test_streamed_small_matches_oracle(small_case):
    _say("streamed vs oracle, 4 views sequential, ragged batches")
    vol = small_case["vol"]
    got = _streamed(small_case["d"], SMALL, small_case["host"], 8, True)
    ref = oracle.deconvolve(vol["stacks"], [p.astype(np.float64) for p in vol["psfs"]], SMALL.iters,
                            update=SMALL.update)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= TOL, f"max|d|/max = {err:.3e}"


@pytest.mark.parametrize("est_host", [False, True], ids=["est_dev", "est_host"])
def test_streamed_given_init(small_case, est_host):
    _say(f"streamed given init est_host={est_host}")
    rng = np.random.default_rng(5)
    init = rng.uniform(50.0, 150.0, small_case["plain"].shape).astype(np.float32)
    ref = _plain(small_case["d"], SMALL, small_case["vol"]["stacks"], init=init)
    got = _streamed(small_case["d"], SMALL, small_case["host"], 8, est_host, init=init)
    np.testing.assert_array_equal(got, ref)


def test_streamed_f32_device_obs():
    """float32 observations already on the device go through the same path."""
    from paper_1503_07998_amd import api

    torch = _torch()
    _say("streamed f32 device stacks, simultaneous, 2 views")
    spec = VolumeSpec("stream_f32", 21, 33, 72, 7, (1.2, 2.5), (0, 90), 30, "f32", 3, "simultaneous", seed=78)
    vol = make_volume(spec, truth=False)
    d = _ctx(spec, vol["psfs"])
    plain = _plain(d, spec, vol["stacks"])
    dev = [torch.from_numpy(s).to("cuda:0") for s in vol["stacks"]]
    got = _streamed(d, spec, dev, 5, False)
    np.testing.assert_array_equal(got, plain)
    with pytest.raises(ValueError):          # pageable host tensors are refused
        api.mvd_deconvolve_stream(d.ctx, [torch.from_numpy(s) for s in vol["stacks"]],
                                  torch.empty(1, device="cuda:0"), api.make_run(21, 1), 5)
    # ... and by the library itself
    from paper_1503_07998_amd import _native as N
    import ctypes
    ptrs = (ctypes.c_void_p * 2)(*[s.ctypes.data for s in vol["stacks"]])
    run = api.make_run(21, 1)
    est = torch.empty((21, 33, 72), device="cuda:0")
    st = N.lib().mvd_deconvolve_stream(d.ctx, ptrs, ctypes.c_void_p(est.data_ptr()), ctypes.byref(run), 5, None)
    assert st == N.MVD_ERR_ARG and "pageable" in api.mvd_last_error(d.ctx)
    d.close()


def test_streamed_full_size_sampled_planes():
    """4 views, 1024 planes of 1024×1024, 41×41 PSFs, 10 sequential iterations,
    uint16 stacks in page-locked host memory, batches of 64 planes (the launch
    configuration the benchmark times).  Planes 0, 517 and 1023 hold rendered
    blob data and are checked against the oracle; every plane is checked for
    the sequential flux identity."""
    torch = _torch()
    spec = CONFIGS["vol1024x4"]
    Z, Y, X = spec.n_z, spec.n_planes, spec.n_x
    sample = [0, 517, 1023]
    _say("full-size streamed run: render sampled planes")
    real = render_planes(spec, sample)
    host = []
    for v in range(spec.n_views):
        t = torch.empty((Z, Y, X), dtype=torch.uint16, pin_memory=True)
        a = t.numpy()
        a[...] = 100
        a[:, :, ::7] = 103             # filler planes: background with a column pattern
        a[:, sample, :] = real[v]
        host.append(t)
    psfs = spec.psfs()
    d = _ctx(spec, psfs)
    _say("full-size streamed run: 1024 planes, batch 64")
    est = _streamed(d, spec, host, 64, False)
    d.close()
    assert np.isfinite(est).all() and est.min() >= 0.0
    last = host[-1].numpy()
    obs_sum = last.sum(axis=(0, 2), dtype=np.float64)          # per plane y
    est_sum = est.sum(axis=(1, 2), dtype=np.float64)
    rel = np.abs(est_sum - obs_sum) / obs_sum
    assert rel.max() <= 1e-5, f"flux identity off by {rel.max():.3e} at plane {rel.argmax()}"
    _say("full-size streamed run: oracle on sampled planes")
    ref = oracle.deconvolve(real, [p.astype(np.float64) for p in psfs], spec.iters, update=spec.update,
                            method="fft")
    for i, y in enumerate(sample):
        err = np.abs(est[y] - ref[i]).max() / np.abs(ref[i]).max()
        assert err <= TOL, f"plane {y}: max|d|/max = {err:.3e}"


def test_streamed_general_update_equals_plain():
    """A normalised run with a low-rank and a full-rank PSF and weight planes
    (the general update: sensitivity planes per batch), streamed in batches
    of 4 of 13 planes: bitwise the device-resident run."""
    from paper_1503_07998_amd import api
    from synthetic import random_psf

    torch = _torch()
    _say("streamed general update, 13 planes, batch 4")
    rng = np.random.default_rng(71)
    Z, Y, X = 28, 13, 36
    p0 = sum(np.outer(rng.uniform(0.05, 1.0, 9), rng.uniform(0.05, 1.0, 9)) for _ in range(2))
    psfs = [(p0 / p0.sum()).astype(np.float32), random_psf(rng, 7, 7).astype(np.float32)]
    d = api.Deconvolver(2, Z, X, 0)
    for v, p in enumerate(psfs):
        d.set_psf(v, p)
    stacks = [rng.uniform(20.0, 400.0, (Z, Y, X)).astype(np.float32) for _ in range(2)]
    planes = [torch.from_numpy(rng.uniform(0.2, 1.0, (Y, Z, X)).astype(np.float32)).to("cuda:0") for _ in range(2)]
    obs = [torch.from_numpy(s).to("cuda:0") for s in stacks]
    est = torch.empty((Y, Z, X), dtype=torch.float32, device="cuda:0")
    run = api.make_run(Y, 3, update="simultaneous", normalize=True, weight_planes=planes)
    nb = api.mvd_workspace_bytes(d.ctx, run)
    ws, run.workspace = _workspace(nb)
    run.workspace_bytes = nb
    api.mvd_deconvolve_planes(d.ctx, obs, est, run)
    torch.cuda.synchronize()
    ref = est.cpu().numpy()
    host = [_pinned(s) for s in stacks]
    est_h = torch.empty((Y, Z, X), dtype=torch.float32, pin_memory=True)
    run = api.make_run(Y, 3, update="simultaneous", normalize=True, weight_planes=planes)
    nb = api.mvd_stream_workspace_bytes(d.ctx, run, 4, True)
    ws2, run.workspace = _workspace(nb)
    run.workspace_bytes = nb
    api.mvd_deconvolve_stream(d.ctx, host, est_h, run, 4)
    torch.cuda.current_stream().synchronize()
    np.testing.assert_array_equal(est_h.numpy(), ref)
    d.close()
