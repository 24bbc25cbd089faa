"""The fused iteration (forward and backward passes of both views in one
launch) against the two-launch form and the oracle.

Every output of the fused kernel is formed by the same operations in the same
order as in the two-launch form, so the estimates (and checkpoints) must be
bitwise equal; each case also checks through the launch timings that the fused
kernel really ran (and did not in the two-launch run), and a few cases are
compared with the oracle directly.  Shapes cover one and several strips per
plane (a partial last strip), row counts that are not a multiple of the row
group, odd and even iteration counts (after an odd count over several strips
ψ^T is copied back from the second plane set), every fused kernel-size bucket, both
observation types and layouts, view weights, checkpoints and plane batches.
"""
import ctypes

import numpy as np
import pytest

import oracle
from synthetic import gaussian_psf

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _torch():
    import torch
    return torch


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _set_tune(spec):
    from paper_1503_07998_amd import _native as N

    lib = N.lib()
    lib.mvd_internal_set_tune.restype = ctypes.c_int
    lib.mvd_internal_set_tune.argtypes = [ctypes.c_char_p]
    lib.mvd_internal_set_tune(spec.encode() if spec is not None else None)


def _case(seed, Y, Z, X, k, dtype, layout):
    rng = np.random.default_rng(seed)
    shape = (Z, Y, X) if layout == "stack_zyx" else (Y, Z, X)
    if dtype == "u16":
        stacks = [rng.integers(50, 3000, shape).astype(np.uint16) for _ in range(2)]
    else:
        stacks = [rng.uniform(10.0, 900.0, shape).astype(np.float32) for _ in range(2)]
    s1 = 0.4 + 0.15 * k
    psfs = [gaussian_psf(k, 1.3, s1).astype(np.float32), gaussian_psf(k, s1, 0.9).astype(np.float32)]
    return stacks, psfs


def _run(stacks, psfs, Y, Z, X, iters, dtype, layout, fused, weights=None, checkpoints=False, batch=0):
    """(ψ^T, checkpoints or None, fused launches, forward launches)."""
    from paper_1503_07998_amd import api

    torch = _torch()
    spec = ["fused=1" if fused else "fused=0"]
    if batch:
        spec.append(f"plane_batch={batch}")
    _set_tune(",".join(spec))
    try:
        ctx = api.mvd_create(2, Z, X, 0)
        try:
            for v in range(2):
                api.mvd_set_psf(ctx, v, psfs[v])
            obs = [torch.from_numpy(np.ascontiguousarray(s)).to("cuda:0") for s in stacks]
            est = torch.empty((Y, Z, X), dtype=torch.float32, device="cuda:0")
            ck = torch.full((iters, Y, Z, X), -1.0, device="cuda:0") if checkpoints else None
            run = api.make_run(Y, iters, obs_dtype=dtype, layout=layout, weights=weights, timing=True,
                               checkpoints=ck.data_ptr() if ck is not None else None)
            nb = api.mvd_workspace_bytes(ctx, run)
            ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda:0")
            run.workspace = (ws.data_ptr() + 255) // 256 * 256
            run.workspace_bytes = nb
            api.mvd_get_timing(ctx, reset=True)
            api.mvd_deconvolve_planes(ctx, obs, est, run)
            torch.cuda.synchronize()
            tim = api.mvd_get_timing(ctx, reset=True)
            return (est.cpu().numpy(), ck.cpu().numpy() if ck is not None else None, tim["fused"][0],
                    tim["forward"][0])
        finally:
            api.mvd_destroy(ctx)
    finally:
        _set_tune(None)


CASES = [
    # seed, Y, Z, X, k, dtype, layout, iters, weights
    (1, 5, 37, 264, 7, "u16", "stack_zyx", 3, None),      # two strips (one partial), odd count
    (2, 3, 64, 64, 15, "f32", "planes_yzx", 2, None),     # one strip: in place
    (3, 4, 100, 520, 31, "u16", "stack_zyx", 10, (0.7, 1.0)),   # three strips, weights
    (4, 2, 8, 256, 3, "f32", "stack_zyx", 1, None),       # one group, one iteration
    (5, 6, 48, 512, 21, "u16", "planes_yzx", 4, None),
    (6, 2, 513, 272, 31, "f32", "stack_zyx", 5, (1.0, 0.4)),   # ragged last group, odd count
    (7, 3, 21, 136, 11, "u16", "stack_zyx", 2, None),
]


@pytest.mark.parametrize("case", CASES, ids=[f"c{c[0]}" for c in CASES])
def test_fused_equals_two_launch(case):
    seed, Y, Z, X, k, dtype, layout, iters, w = case
    _say(f"fused vs two-launch: Y={Y} Z={Z} X={X} K={k} {dtype} {layout} T={iters} w={w}")
    stacks, psfs = _case(seed, Y, Z, X, k, dtype, layout)
    got, _, nf, _ = _run(stacks, psfs, Y, Z, X, iters, dtype, layout, True, weights=w)
    ref, _, nf0, nfw0 = _run(stacks, psfs, Y, Z, X, iters, dtype, layout, False, weights=w)
    assert nf == iters, nf
    assert nf0 == 0 and nfw0 > 0
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("case", [CASES[0], CASES[2], CASES[5]], ids=["c1", "c3", "c6"])
def test_fused_matches_oracle(case):
    seed, Y, Z, X, k, dtype, layout, iters, w = case
    _say(f"fused vs oracle: Y={Y} Z={Z} X={X} K={k} T={iters}")
    stacks, psfs = _case(seed, Y, Z, X, k, dtype, layout)
    got, _, nf, _ = _run(stacks, psfs, Y, Z, X, iters, dtype, layout, True, weights=w)
    assert nf > 0
    ys = [0, Y - 1]
    sub = [s[:, ys, :] if layout == "stack_zyx" else s[ys] for s in stacks]
    ref = oracle.deconvolve(sub, [p.astype(np.float64) for p in psfs], iters, layout=layout,
                            weights=w, method="fft" if Z * X > 20000 else "direct")
    e = np.abs(got[ys] - ref).max() / np.abs(ref).max()
    assert e <= TOL, e


def test_fused_checkpoints_and_batches():
    """Checkpoints ψ^0..ψ^{T−1} and plane batches: bitwise the two-launch run's."""
    Y, Z, X, k, iters = 7, 40, 264, 15, 3
    _say("fused: checkpoints, plane batches of 3")
    stacks, psfs = _case(11, Y, Z, X, k, "u16", "stack_zyx")
    got, ck, nf, _ = _run(stacks, psfs, Y, Z, X, iters, "u16", "stack_zyx", True, checkpoints=True)
    ref, ck0, _, _ = _run(stacks, psfs, Y, Z, X, iters, "u16", "stack_zyx", False, checkpoints=True)
    assert nf == iters          # with checkpoints every iteration fuses (the slots alternate)
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(ck, ck0)
    gb, _, nfb, _ = _run(stacks, psfs, Y, Z, X, iters, "u16", "stack_zyx", True, batch=3)
    assert nfb == 3 * iters         # three batches
    np.testing.assert_array_equal(gb, ref)


def test_fused_not_taken_where_it_does_not_apply():
    """41-tap kernels, sequential updates and the periodic boundary run the
    two-launch passes (no fused launch) even where fused launches are asked for."""
    from paper_1503_07998_amd import api

    torch = _torch()
    _say("fused: fallbacks")
    Y, Z, X = 2, 48, 64
    stacks, psf41 = _case(21, Y, Z, X, 41, "f32", "stack_zyx")
    _, psf15 = _case(21, Y, Z, X, 15, "f32", "stack_zyx")
    ctx = api.mvd_create(2, Z, X, 0)
    _set_tune("fused=1")
    try:
        obs = [torch.from_numpy(s).to("cuda:0") for s in stacks]
        est = torch.empty((Y, Z, X), device="cuda:0")
        for psfs, kw in ((psf41, {}), (psf15, {"update": "sequential"}), (psf15, {"boundary": "periodic"})):
            for v in range(2):
                api.mvd_set_psf(ctx, v, psfs[v])
            run = api.make_run(Y, 2, obs_dtype="f32", timing=True, **kw)
            nb = api.mvd_workspace_bytes(ctx, run)
            ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda:0")
            run.workspace = (ws.data_ptr() + 255) // 256 * 256
            run.workspace_bytes = nb
            api.mvd_get_timing(ctx, reset=True)
            api.mvd_deconvolve_planes(ctx, obs, est, run)
            torch.cuda.synchronize()
            tim = api.mvd_get_timing(ctx, reset=True)
            assert tim["fused"][0] == 0 and tim["forward"][0] > 0, kw
    finally:
        _set_tune(None)
        api.mvd_destroy(ctx)


def test_tuner_times_the_fused_form():
    """A tuned run of a fused-eligible workload times the fused candidate too:
    whichever form it keeps, the result is within float32 rounding of the
    untuned two-launch run (tuned shapes change summation orders only)."""
    Y, Z, X, k = 4, 64, 264, 7
    _say("tuner with the fused candidate")
    stacks, psfs = _case(31, Y, Z, X, k, "u16", "stack_zyx")
    ref, _, _, _ = _run(stacks, psfs, Y, Z, X, 4, "u16", "stack_zyx", False)
    from paper_1503_07998_amd import api

    torch = _torch()
    ctx = api.mvd_create(2, Z, X, 0)
    try:
        for v in range(2):
            api.mvd_set_psf(ctx, v, psfs[v])
        obs = [torch.from_numpy(np.ascontiguousarray(s)).to("cuda:0") for s in stacks]
        est = torch.empty((Y, Z, X), device="cuda:0")
        run = api.make_run(Y, 4, obs_dtype="u16", tune=True, timing=True)
        nb = api.mvd_workspace_bytes(ctx, run)
        ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda:0")
        run.workspace = (ws.data_ptr() + 255) // 256 * 256
        run.workspace_bytes = nb
        api.mvd_deconvolve_planes(ctx, obs, est, run)
        torch.cuda.synchronize()
        tim = api.mvd_get_timing(ctx, reset=True)
        assert tim["fused"][0] in (0, 4)
        got = est.cpu().numpy()
    finally:
        api.mvd_destroy(ctx)
    e = np.abs(got - ref).max() / np.abs(ref).max()
    assert e <= 1e-5, e
