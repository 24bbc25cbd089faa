"""The allocation-free entry point against the ordinary one.

mvd_deconvolve_planes_static takes its workspace from a static per-device
scratch array instead of the caller's buffer and runs the volume in batches
of planes that fit it.  Its estimate must equal mvd_deconvolve_planes' bitwise
(the same kernels and per-pixel arithmetic), on two calls in a row, the second
with a smaller input, and also when the scratch holds fewer planes than the
volume (several batches).
"""
import numpy as np
import pytest

from synthetic import gaussian_psf, random_psf

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _run_both(nz, nx, ny, views, k, iters, update, seed, obs_dtype="u16"):
    import torch

    from paper_1503_07998_amd import _native as N
    from paper_1503_07998_amd import api

    rng = np.random.default_rng(seed)
    if obs_dtype == "u16":
        stacks = [rng.integers(50, 3000, (nz, ny, nx)).astype(np.uint16) for _ in range(views)]
    else:
        stacks = [rng.uniform(50.0, 3000.0, (nz, ny, nx)).astype(np.float32) for _ in range(views)]
    psfs = [gaussian_psf(k, 1.5 + 0.7 * v, 4.0 - 0.5 * v) for v in range(views)]
    psfs[-1] = random_psf(rng, k, k, separable=True)
    ctx = api.mvd_create(views, nz, nx, 0)
    try:
        for v in range(views):
            api.mvd_set_psf(ctx, v, psfs[v])
        obs = [torch.from_numpy(s).to("cuda:0") for s in stacks]
        run = api.make_run(ny, iters, update=update, obs_dtype=obs_dtype)
        nbytes = api.mvd_workspace_bytes(ctx, run)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda:0")
        run.workspace = (ws.data_ptr() + 255) // 256 * 256
        run.workspace_bytes = nbytes
        ref = torch.empty((ny, nz, nx), dtype=torch.float32, device="cuda:0")
        api.mvd_deconvolve_planes(ctx, obs, ref, run)
        torch.cuda.synchronize()
        run.workspace = None
        run.workspace_bytes = 0
        got = torch.full((ny, nz, nx), -1.0, dtype=torch.float32, device="cuda:0")
        api.mvd_deconvolve_planes_static(ctx, obs, got, run)
        torch.cuda.synchronize()
        one = api.make_run(1, iters, update=update, obs_dtype=obs_dtype)
        batches = -(-ny // max(1, N.MVD_SCRATCH_BYTES // api.mvd_workspace_bytes(ctx, one)))
        return ref.cpu().numpy(), got.cpu().numpy(), batches
    finally:
        api.mvd_destroy(ctx)


def test_static_entry_point_matches_the_workspace_one():
    """Two calls in a row on one GPU, the second smaller; the first needs several
    batches of planes (512×512 planes, 2 views: 4 MiB of workspace per plane)."""
    _say("static scratch: 40 planes of 512x512, 2 views, K 31, 3 its (several batches)")
    ref, got, nb = _run_both(512, 512, 40, 2, 31, 3, "simultaneous", 1)
    assert nb > 1
    np.testing.assert_array_equal(got, ref)
    _say("static scratch: 7 planes of 72x96, 3 views, K 15, 4 sequential its (smaller input)")
    ref, got, nb = _run_both(72, 96, 7, 3, 15, 4, "sequential", 2, obs_dtype="f32")
    assert nb == 1
    np.testing.assert_array_equal(got, ref)


def test_static_entry_point_refuses_a_workspace_and_event_flags():
    import torch

    from paper_1503_07998_amd import _native as N
    from paper_1503_07998_amd import api

    _say("static scratch: argument checks")
    ctx = api.mvd_create(1, 16, 16, 0)
    try:
        api.mvd_set_psf(ctx, 0, gaussian_psf(5, 1.0, 1.0))
        obs = [torch.ones((16, 2, 16), dtype=torch.float32, device="cuda:0")]
        est = torch.empty((2, 16, 16), dtype=torch.float32, device="cuda:0")
        ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
        run = api.make_run(2, 1)
        run.workspace = (ws.data_ptr() + 255) // 256 * 256
        run.workspace_bytes = 1 << 16
        with pytest.raises(N.MvdError) as e:
            api.mvd_deconvolve_planes_static(ctx, obs, est, run)
        assert e.value.status == N.MVD_ERR_ARG
        for kw in ({"timing": True}, {"graph": True}, {"tune": True}):
            run = api.make_run(2, 1, **kw)
            with pytest.raises(N.MvdError) as e:
                api.mvd_deconvolve_planes_static(ctx, obs, est, run)
            assert e.value.status == N.MVD_ERR_ARG
    finally:
        api.mvd_destroy(ctx)
