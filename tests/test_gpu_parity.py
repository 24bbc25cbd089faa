"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar: max|Δ| / max|oracle| ≤ 1e-4 after the stated iterations (float32 path,
float64 oracle); bitwise for the reslice, the delta-PSF fixed point and the
run-to-run invariances (determinism, resume, plane subsets, checkpoints).
Every case prints its name before it touches the GPU.
"""
import zlib

import numpy as np
import pytest

import oracle
from synthetic import CONFIGS, gaussian_psf, make_volume, random_psf

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _torch():
    import torch
    return torch


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def gpu_run(stacks, psfs, iters, layout="stack_zyx", **kw):
    from paper_1503_07998_amd import deconvolve

    torch = _torch()
    obs = [_dev(s) for s in stacks]
    if "est" in kw and isinstance(kw["est"], np.ndarray):
        kw["est"] = _dev(kw["est"].astype(np.float32))
    out = deconvolve(obs, psfs, iters=iters, layout=layout, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def oracle_run(stacks, psfs, iters, layout="stack_zyx", method=None, **kw):
    kw = dict(kw)
    if "est" in kw:
        kw["init_given"] = kw.pop("est")
    kw.pop("force_2d", None)
    if "back" in kw and kw.get("back") == "explicit":
        kw["back_taps"] = [np.asarray(x, dtype=np.float64) for x in kw["back_taps"]]
    if method is None:
        shp = stacks[0].shape
        area = shp[0] * shp[2] if layout == "stack_zyx" else shp[1] * shp[2]
        k2 = max(p.shape[0] * p.shape[1] for p in psfs)
        method = "fft" if area * k2 > 2e6 else "direct"
    ps = [np.asarray(p, dtype=np.float64) for p in psfs]
    return oracle.deconvolve(stacks, ps, iters, layout=layout, method=method, **kw)


def rel_err(got, ref):
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def check(got, ref, tol=TOL):
    assert np.all(np.isfinite(got))
    e = rel_err(got, ref)
    assert e <= tol, f"max|d|/max = {e:.3e} > {tol}"
    return e


# ---------------------------------------------------------------------------
# Reslice
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["u16", "f32"])
@pytest.mark.parametrize("shape", [(5, 7, 9), (33, 3, 128), (2, 1, 1), (17, 64, 30)])
def test_reslice_bitwise(dtype, shape):
    from paper_1503_07998_amd import api

    torch = _torch()
    _say(f"reslice {dtype} {shape}")
    rng = np.random.default_rng(1)
    if dtype == "u16":
        st = rng.integers(0, 65536, size=shape, dtype=np.uint16)
    else:
        st = rng.normal(50.0, 80.0, size=shape).astype(np.float32)
        st.flat[::7] = np.nan
    nz, ny, nx = shape
    ctx = api.mvd_create(1, nz, nx, 0)
    try:
        d = _dev(st)
        out = torch.empty((ny, nz, nx), dtype=torch.float32, device="cuda:0")
        api.mvd_reslice(ctx, d, ny, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    finally:
        api.mvd_destroy(ctx)
    ref = oracle.reslice(st).astype(np.float32)
    np.testing.assert_array_equal(got, ref)


# ---------------------------------------------------------------------------
# Small configuration (2 views, 32 planes of 128×128, 15×15, 10 iterations)
# ---------------------------------------------------------------------------
def test_small_config_all_planes():
    _say("small config, all planes, simultaneous, zero")
    spec = CONFIGS["small"]
    vol = make_volume(spec)
    got = gpu_run(vol["stacks"], vol["psfs"], spec.iters)
    ref = oracle_run(vol["stacks"], vol["psfs"], spec.iters)
    check(got, ref)


@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_small_config_modes(update, boundary):
    _say(f"small config 8 planes {update} {boundary}")
    spec = CONFIGS["small"]
    vol = make_volume(spec, planes=8)
    got = gpu_run(vol["stacks"], vol["psfs"], 10, update=update, boundary=boundary)
    ref = oracle_run(vol["stacks"], vol["psfs"], 10, update=update, boundary=boundary)
    check(got, ref)


# ---------------------------------------------------------------------------
# Ragged shapes, asymmetric kernels, both kernel families
# ---------------------------------------------------------------------------
CASES = [
    # (Y, Z, X, kernel shapes, separable, boundary, update, weights)
    (3, 8, 8, [(3, 5), (5, 3)], True, "zero", "simultaneous", None),
    (3, 8, 8, [(3, 5), (5, 3)], False, "periodic", "simultaneous", None),
    (2, 1, 37, [(1, 9), (3, 3)], True, "zero", "sequential", None),
    (2, 41, 1, [(9, 1), (3, 3)], True, "periodic", "simultaneous", None),
    (2, 8, 8, [(15, 15), (11, 13)], True, "zero", "simultaneous", [1.0, 0.6]),
    (2, 8, 8, [(15, 15), (11, 13)], False, "periodic", "sequential", [0.7, 1.0]),
    (4, 37, 53, [(7, 5), (5, 9), (3, 3)], True, "zero", "sequential", [1.0, 0.5, 0.25]),
    (4, 37, 53, [(7, 5), (5, 9), (3, 3)], False, "zero", "simultaneous", None),
    (2, 70, 100, [(31, 31), (31, 31)], True, "zero", "simultaneous", None),
    (2, 70, 100, [(21, 41), (41, 21)], True, "periodic", "simultaneous", None),
    (2, 13, 200, [(63, 63)], True, "zero", "simultaneous", None),
    (2, 24, 700, [(31, 31), (31, 31)], True, "zero", "simultaneous", None),     # 2 columns/thread
    (2, 24, 700, [(41, 41), (41, 41)], True, "periodic", "sequential", None),
    (2, 16, 1100, [(9, 9), (9, 9)], True, "zero", "simultaneous", None),        # strips with halo
    (2, 16, 1100, [(9, 9), (9, 9)], True, "periodic", "simultaneous", None),
    (1, 12, 600, [(63, 63)], True, "periodic", "simultaneous", None),           # strips, K=63
    (2, 9, 66, [(5, 5), (7, 7)], False, "zero", "simultaneous", [0.0, 1.0]),
]


@pytest.mark.parametrize("case", CASES, ids=[f"c{i}" for i in range(len(CASES))])
def test_ragged_cases(case):
    Y, Z, X, shapes, sep, boundary, update, weights = case
    _say(f"ragged Y={Y} Z={Z} X={X} k={shapes} sep={sep} {boundary} {update} w={weights}")
    rng = np.random.default_rng(zlib.crc32(repr(case).encode()))
    psfs = [random_psf(rng, kz, kx, separable=sep).astype(np.float32) for kz, kx in shapes]
    stacks = [rng.uniform(0.0, 200.0, (Z, Y, X)).astype(np.float32) for _ in shapes]
    got = gpu_run(stacks, psfs, 5, boundary=boundary, update=update, weights=weights)
    ref = oracle_run(stacks, psfs, 5, boundary=boundary, update=update, weights=weights)
    check(got, ref)


def test_separable_and_general_kernels_agree():
    _say("force 2D vs separable")
    spec = CONFIGS["small"]
    vol = make_volume(spec, planes=4)
    a = gpu_run(vol["stacks"], vol["psfs"], 10)
    b = gpu_run(vol["stacks"], vol["psfs"], 10, force_2d=True)
    # two float32 summation orders (two 1D passes vs K² taps), ~1e-7 per
    # convolution, compounded over 40 convolutions of the multiplicative update
    assert rel_err(a, b) <= 1e-5


@pytest.mark.parametrize("back", ["efficient_bayes", "opt1", "opt2"])
def test_compound_back_projectors(back):
    _say(f"compound {back}")
    spec = CONFIGS["small"]
    vol = make_volume(spec, planes=4)
    got = gpu_run(vol["stacks"], vol["psfs"], 6, back=back)
    ref = oracle_run(vol["stacks"], vol["psfs"], 6, back=back)
    check(got, ref)


def test_compound_back_projector_non_separable():
    _say("compound efficient_bayes, asymmetric non-separable PSFs")
    rng = np.random.default_rng(8)
    psfs = [random_psf(rng, 7, 5).astype(np.float32), random_psf(rng, 5, 7).astype(np.float32)]
    stacks = [rng.uniform(10.0, 200.0, (20, 3, 24)).astype(np.float32) for _ in range(2)]
    got = gpu_run(stacks, psfs, 4, back="efficient_bayes")
    ref = oracle_run(stacks, psfs, 4, back="efficient_bayes")
    check(got, ref)


def test_explicit_back_projector():
    _say("explicit back-projector")
    rng = np.random.default_rng(9)
    psfs = [random_psf(rng, 5, 5, separable=True).astype(np.float32) for _ in range(2)]
    backs = [random_psf(rng, 5, 5).astype(np.float32) for _ in range(2)]
    stacks = [rng.uniform(10.0, 200.0, (16, 2, 16)).astype(np.float32) for _ in range(2)]
    got = gpu_run(stacks, psfs, 3, back="explicit", back_taps=backs)
    ref = oracle_run(stacks, psfs, 3, back="explicit", back_taps=backs)
    check(got, ref)


# ---------------------------------------------------------------------------
# Exact properties
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
def test_delta_psf_fixed_point_bitwise(update):
    _say(f"delta PSF fixed point {update}")
    rng = np.random.default_rng(10)
    phi = rng.uniform(1.0, 500.0, (9, 3, 40)).astype(np.float32)
    d = np.zeros((3, 5), dtype=np.float32)
    d[1, 2] = 1.0
    got = gpu_run([phi, phi], [d, d], 7, update=update)
    np.testing.assert_array_equal(got.astype(np.float32), oracle.reslice(phi).astype(np.float32))


def test_init_modes_and_zero_iterations():
    _say("init modes")
    rng = np.random.default_rng(11)
    psfs = [random_psf(rng, 5, 5, separable=True).astype(np.float32) for _ in range(2)]
    stacks = [rng.uniform(10.0, 200.0, (16, 3, 20)).astype(np.float32) for _ in range(2)]
    mean = gpu_run(stacks, psfs, 0)
    np.testing.assert_allclose(mean, oracle_run(stacks, psfs, 0), rtol=1e-7)
    c = gpu_run(stacks, psfs, 0, init="const", init_const=3.5)
    assert np.all(c == 3.5)
    given = rng.uniform(5.0, 50.0, (3, 16, 20)).astype(np.float32)
    g0 = gpu_run(stacks, psfs, 0, init="given", est=given)
    np.testing.assert_array_equal(g0.astype(np.float32), given)
    got = gpu_run(stacks, psfs, 4, init="given", est=given)
    check(got, oracle_run(stacks, psfs, 4, init="given", est=given.astype(np.float64)))
    got = gpu_run(stacks, psfs, 4, init="const", init_const=2.0)
    check(got, oracle_run(stacks, psfs, 4, init="const", init_const=2.0))


@pytest.mark.parametrize("dtype", ["u16", "f32"])
@pytest.mark.parametrize("layout", ["stack_zyx", "planes_yzx"])
def test_dtypes_and_layouts(dtype, layout):
    _say(f"dtype {dtype} layout {layout}")
    rng = np.random.default_rng(12)
    psfs = [gaussian_psf(9, 1.5, 3.0).astype(np.float32), gaussian_psf(9, 3.0, 1.5).astype(np.float32)]
    shape = (24, 5, 40) if layout == "stack_zyx" else (5, 24, 40)
    if dtype == "u16":
        stacks = [rng.integers(0, 2000, size=shape, dtype=np.uint16) for _ in range(2)]
    else:
        stacks = [rng.normal(100.0, 60.0, size=shape).astype(np.float32) for _ in range(2)]
    got = gpu_run(stacks, psfs, 5, layout=layout)
    ref = oracle_run(stacks, psfs, 5, layout=layout)
    check(got, ref)


@pytest.mark.parametrize("shape", [(24, 5, 40), (13, 3, 37), (9, 4, 66), (40, 2, 8)],
                         ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
def test_observation_forms_bitwise(shape, update):
    """The forward passes read the observations in place (uint16 or float32,
    stack or plane layout, 16-byte or element-wise accesses): the same values
    in any of the four forms give bitwise the same estimate."""
    _say(f"observation forms {shape} {update}")
    rng = np.random.default_rng(31)
    psfs = [gaussian_psf(7, 1.2, 2.5).astype(np.float32), gaussian_psf(7, 2.5, 1.2).astype(np.float32)]
    stacks = [rng.integers(0, 3000, size=shape, dtype=np.uint16) for _ in range(2)]
    planes = [np.ascontiguousarray(np.transpose(s, (1, 0, 2))) for s in stacks]
    ref = gpu_run(stacks, psfs, 3, update=update)
    for obs, layout in (([s.astype(np.float32) for s in stacks], "stack_zyx"), (planes, "planes_yzx"),
                        ([p.astype(np.float32) for p in planes], "planes_yzx")):
        got = gpu_run(obs, psfs, 3, layout=layout, update=update)
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("batch", [1, 3, 7])
@pytest.mark.parametrize("update,layout,dtype", [("simultaneous", "stack_zyx", "u16"),
                                                  ("sequential", "planes_yzx", "f32"),
                                                  ("simultaneous", "planes_yzx", "u16")])
def test_plane_batches_bitwise(batch, update, layout, dtype):
    """Planes are independent: running the volume batch by batch of planes
    (each batch through every iteration) gives bitwise the whole-volume
    result, with checkpoints at the same slots, for the mean, given and
    constant initial estimates."""
    import ctypes
    from paper_1503_07998_amd import _native as N

    torch = _torch()
    _say(f"plane batches of {batch}: {update} {layout} {dtype}")
    rng = np.random.default_rng(41)
    psfs = [gaussian_psf(9, 1.5, 3.0).astype(np.float32), gaussian_psf(9, 3.0, 1.5).astype(np.float32)]
    shape = (20, 9, 32) if layout == "stack_zyx" else (9, 20, 32)
    if dtype == "u16":
        obs = [rng.integers(0, 2000, size=shape, dtype=np.uint16) for _ in range(2)]
    else:
        obs = [rng.uniform(0.0, 500.0, size=shape).astype(np.float32) for _ in range(2)]
    lib = N.lib()
    lib.mvd_internal_set_tune.argtypes = [ctypes.c_char_p]

    given = rng.uniform(10.0, 100.0, (9, 20, 32)).astype(np.float32)

    def run():
        from paper_1503_07998_amd import Deconvolver

        d = Deconvolver(2, 20, 32, 0)
        for v, p in enumerate(psfs):
            d.set_psf(v, p)
        ck = torch.empty((4, 9, 20, 32), dtype=torch.float32, device="cuda:0")
        a = d.run([_dev(o) for o in obs], iters=4, update=update, layout=layout).cpu().numpy()
        b = d.run([_dev(o) for o in obs], iters=4, update=update, layout=layout, checkpoints=ck).cpu().numpy()
        g = d.run([_dev(o) for o in obs], iters=3, update=update, layout=layout, init="given",
                  est=_dev(given)).cpu().numpy()
        c = d.run([_dev(o) for o in obs], iters=2, update=update, layout=layout, init="const",
                  init_const=7.0).cpu().numpy()
        d.close()
        return a, b, ck.cpu().numpy(), g, c

    try:
        lib.mvd_internal_set_tune(b"")
        ref = run()
        lib.mvd_internal_set_tune(f"plane_batch={batch}".encode())
        got = run()
    finally:
        lib.mvd_internal_set_tune(None)
    for x, y in zip(got, ref):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("x,k,update", [(600, 41, "sequential"), (1000, 31, "simultaneous"), (1024, 41, "simultaneous")])
def test_wide_rows_bitwise(x, k, update):
    """Rows of 513–1024 columns as one column per thread in up to 1024-thread
    work-groups give bitwise the results of the two-columns-per-thread form."""
    import ctypes
    from paper_1503_07998_amd import _native as N

    _say(f"wide rows X={x} K={k} {update}")
    rng = np.random.default_rng(x + k)
    psfs = [gaussian_psf(k, 1.5, k / 5.0).astype(np.float32), gaussian_psf(k, k / 5.0, 1.5).astype(np.float32)]
    obs = [rng.integers(0, 3000, size=(24, 3, x), dtype=np.uint16) for _ in range(2)]
    lib = N.lib()
    lib.mvd_internal_set_tune.argtypes = [ctypes.c_char_p]
    try:
        lib.mvd_internal_set_tune(b"wide=2")
        ref = gpu_run(obs, psfs, 3, update=update)
        lib.mvd_internal_set_tune(b"")
        got = gpu_run(obs, psfs, 3, update=update)
    finally:
        lib.mvd_internal_set_tune(None)
    np.testing.assert_array_equal(got, ref)


NORM_CASES = [
    # (Z, Y, X, kernel shapes, update, boundary, weights)
    (37, 3, 45, [(9, 7), (7, 9)], "simultaneous", "zero", None),           # ragged, element-wise
    (40, 4, 64, [(15, 15), (11, 11)], "simultaneous", "zero", [0.8, 0.6]),  # split-view backward
    (33, 2, 48, [(9, 5), (5, 9), (3, 3)], "sequential", "zero", [1.0, 0.5, 0.9]),
    (24, 2, 40, [(7, 7), (9, 9)], "simultaneous", "periodic", None),
    (20, 2, 600, [(31, 31), (21, 21)], "sequential", "zero", None),        # rows wider than 512
    (16, 3, 32, [(31, 31)], "simultaneous", "zero", None),                 # kernel taller than the plane
]


@pytest.mark.parametrize("case", NORM_CASES, ids=[f"n{i}" for i in range(len(NORM_CASES))])
def test_normalized_matches_oracle(case):
    """EM-normalised back-projection (MVD_FLAG_NORMALIZE) against the oracle's
    normalised update."""
    Z, Y, X, shapes, update, boundary, weights = case
    _say(f"normalised Z={Z} Y={Y} X={X} k={shapes} {update} {boundary} w={weights}")
    rng = np.random.default_rng(Z * 100 + X)
    psfs = [random_psf(rng, kz, kx, separable=True).astype(np.float32) for kz, kx in shapes]
    stacks = [rng.integers(0, 3000, size=(Z, Y, X), dtype=np.uint16) for _ in shapes]
    got = gpu_run(stacks, psfs, 4, update=update, boundary=boundary, weights=weights, normalize=True)
    ref = oracle_run(stacks, psfs, 4, update=update, boundary=boundary, weights=weights, normalize=True)
    check(got, ref)
    if boundary == "zero":   # the normalisation changes the result near the edges
        plain = oracle_run(stacks, psfs, 4, update=update, boundary=boundary, weights=weights)
        assert np.abs(plain - ref).max() > 1e-3 * np.abs(ref).max()


WPL_CASES = [
    # (Z, Y, X, kernel shapes, update, scalar weights, normalize)
    (40, 3, 64, [(15, 15), (11, 11)], "simultaneous", None, False),
    (37, 2, 45, [(9, 7), (7, 9), (5, 5)], "sequential", [0.9, 0.7, 1.0], False),
    (24, 2, 600, [(21, 21), (9, 9)], "simultaneous", [0.8, 1.0], True),
]


@pytest.mark.parametrize("case", WPL_CASES, ids=[f"w{i}" for i in range(len(WPL_CASES))])
def test_weight_planes_match_oracle(case):
    """Per-pixel view weights ω_v (times the scalar weights) against the
    oracle's per-pixel tempering."""
    torch = _torch()
    Z, Y, X, shapes, update, weights, normalize = case
    _say(f"weight planes Z={Z} Y={Y} X={X} k={shapes} {update} w={weights} normalize={normalize}")
    rng = np.random.default_rng(Z * 10 + X)
    psfs = [random_psf(rng, kz, kx, separable=True).astype(np.float32) for kz, kx in shapes]
    stacks = [rng.integers(0, 3000, size=(Z, Y, X), dtype=np.uint16) for _ in shapes]
    om = [rng.uniform(0.0, 1.0, (Y, Z, X)).astype(np.float32) for _ in shapes]
    planes = [torch.from_numpy(o).to("cuda:0") for o in om]
    got = gpu_run(stacks, psfs, 3, update=update, weights=weights, normalize=normalize, weight_planes=planes)
    ws = [1.0] * len(shapes) if weights is None else weights
    eff = [np.float32(w) * o.astype(np.float64) for w, o in zip(ws, om)]
    ref = oracle_run(stacks, psfs, 3, update=update, weights=eff, normalize=normalize)
    check(got, ref)


GENERAL_CASES = [
    # (Z, Y, X, [(kz, kx, rank: 1 separable, 0 full, r low)], update, boundary, normalize, planes, force_2d)
    (40, 3, 52, [(9, 9, 3), (7, 7, 1)], "simultaneous", "zero", True, False, False),
    (33, 2, 45, [(9, 9, 0), (5, 7, 1)], "sequential", "zero", True, True, False),
    (28, 2, 40, [(11, 11, 2), (9, 9, 0)], "simultaneous", "periodic", False, True, False),
    (26, 2, 38, [(9, 7, 1), (7, 9, 1)], "sequential", "zero", True, True, True),
    (35, 2, 61, [(31, 31, 0)], "simultaneous", "zero", True, False, False),
]


def _psf_of(rng, kz, kx, rank):
    if rank == 1:
        return random_psf(rng, kz, kx, separable=True).astype(np.float32)
    if rank == 0:
        return random_psf(rng, kz, kx).astype(np.float32)
    p = sum(np.outer(rng.uniform(0.05, 1.0, kz), rng.uniform(0.05, 1.0, kx)) for _ in range(rank))
    return (p / p.sum()).astype(np.float32)


@pytest.mark.parametrize("case", GENERAL_CASES, ids=[f"g{i}" for i in range(len(GENERAL_CASES))])
def test_general_update_matches_oracle(case):
    """Per-pixel weights and the EM-normalised back-projection with
    back-projectors that are not rank one (sums of terms, K×K) or with the
    K×K passes forced: each view's back-projection is stored and ψ updated
    pointwise, with the sensitivity 1 ⊛ X_v computed by the same pass."""
    torch = _torch()
    Z, Y, X, shapes, update, boundary, normalize, with_planes, force_2d = case
    _say(f"general update Z={Z} Y={Y} X={X} k={shapes} {update} {boundary} normalize={normalize} "
         f"planes={with_planes} force_2d={force_2d}")
    rng = np.random.default_rng(Z * 17 + X)
    psfs = [_psf_of(rng, kz, kx, r) for kz, kx, r in shapes]
    stacks = [rng.uniform(10.0, 400.0, (Z, Y, X)).astype(np.float32) for _ in shapes]
    kw = dict(update=update, boundary=boundary, normalize=normalize)
    if with_planes:
        om = [rng.uniform(0.2, 1.0, (Y, Z, X)).astype(np.float32) for _ in shapes]
        got = gpu_run(stacks, psfs, 3, weight_planes=[torch.from_numpy(o).to("cuda:0") for o in om],
                      force_2d=force_2d, **kw)
        ref = oracle_run(stacks, psfs, 3, weights=[o.astype(np.float64) for o in om], method="direct", **kw)
    else:
        got = gpu_run(stacks, psfs, 3, weights=[0.9] * len(shapes), force_2d=force_2d, **kw)
        ref = oracle_run(stacks, psfs, 3, weights=[0.9] * len(shapes), method="direct", **kw)
    check(got, ref)


def test_unit_weight_planes_are_scalar_weights_bitwise():
    """Planes of ones leave the scalar weights: bitwise the scalar-weighted run
    (which takes the split-view backward; the weighted one the two-plane form)."""
    torch = _torch()
    _say("unit weight planes vs scalar weights")
    rng = np.random.default_rng(97)
    psfs = [gaussian_psf(15, 1.5, 3.0).astype(np.float32), gaussian_psf(15, 3.0, 1.5).astype(np.float32)]
    stacks = [rng.integers(0, 3000, size=(48, 3, 64), dtype=np.uint16) for _ in range(2)]
    ones = [torch.ones((3, 48, 64), dtype=torch.float32, device="cuda:0") for _ in range(2)]
    a = gpu_run(stacks, psfs, 4, weights=[0.8, 0.6])
    b = gpu_run(stacks, psfs, 4, weights=[0.8, 0.6], weight_planes=ones)
    np.testing.assert_array_equal(a, b)


def test_weight_planes_graph_replays():
    """A captured run is keyed by its weight planes too: replays with other
    planes equal the eager runs with them."""
    from paper_1503_07998_amd import api

    torch = _torch()
    _say("weight planes under graph replay")
    rng = np.random.default_rng(99)
    Z, Y, X = 24, 3, 40
    d = api.Deconvolver(2, Z, X, 0)
    for v in range(2):
        d.set_psf(v, gaussian_psf(9, 1.5 + v, 3.0 - v).astype(np.float32))
    obs = [torch.from_numpy(rng.integers(0, 3000, size=(Z, Y, X), dtype=np.uint16)).to("cuda:0") for _ in range(2)]
    sets = [[torch.from_numpy(rng.uniform(0.2, 1.0, (Y, Z, X)).astype(np.float32)).to("cuda:0") for _ in range(2)]
            for _ in range(2)]
    est = torch.empty((Y, Z, X), dtype=torch.float32, device="cuda:0")
    outs = {}
    for graph in (False, True):
        for i, planes in enumerate(sets):
            run = api.make_run(Y, 3, obs_dtype="u16", graph=graph, weight_planes=planes)
            nb = api.mvd_workspace_bytes(d.ctx, run)
            ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda:0")
            run.workspace = (ws.data_ptr() + 255) // 256 * 256
            run.workspace_bytes = nb
            for _ in range(2 if graph else 1):
                api.mvd_deconvolve_planes(d.ctx, obs, est, run)
                torch.cuda.synchronize()
            outs[(graph, i)] = est.cpu().numpy().copy()
            del ws
    d.close()
    for i in range(2):
        np.testing.assert_array_equal(outs[(True, i)], outs[(False, i)])
    assert np.abs(outs[(False, 0)] - outs[(False, 1)]).max() > 0


def test_weight_planes_in_plane_batches_bitwise():
    import ctypes
    from paper_1503_07998_amd import _native as N

    torch = _torch()
    _say("weight planes with plane batches")
    rng = np.random.default_rng(98)
    psfs = [gaussian_psf(9, 1.5, 3.0).astype(np.float32), gaussian_psf(9, 3.0, 1.5).astype(np.float32)]
    stacks = [rng.integers(0, 3000, size=(20, 7, 32), dtype=np.uint16) for _ in range(2)]
    planes = [torch.from_numpy(rng.uniform(0.0, 1.0, (7, 20, 32)).astype(np.float32)).to("cuda:0") for _ in range(2)]
    lib = N.lib()
    lib.mvd_internal_set_tune.argtypes = [ctypes.c_char_p]
    try:
        lib.mvd_internal_set_tune(b"")
        a = gpu_run(stacks, psfs, 3, weight_planes=planes)
        lib.mvd_internal_set_tune(b"plane_batch=3")
        b = gpu_run(stacks, psfs, 3, weight_planes=planes)
    finally:
        lib.mvd_internal_set_tune(None)
    np.testing.assert_array_equal(a, b)


def test_division_guard():
    _say("division guard")
    rng = np.random.default_rng(13)
    psfs = [random_psf(rng, 3, 3, separable=True).astype(np.float32) for _ in range(2)]
    stacks = [rng.uniform(1.0, 100.0, (12, 2, 30)).astype(np.float32) for _ in range(2)]
    given = rng.uniform(1.0, 10.0, (2, 12, 30)).astype(np.float32)
    given[:, :, :12] = 0.0
    got = gpu_run(stacks, psfs, 3, init="given", est=given)
    ref = oracle_run(stacks, psfs, 3, init="given", est=given.astype(np.float64))
    check(got, ref)


def test_determinism_resume_subset_checkpoints():
    from paper_1503_07998_amd import Deconvolver

    torch = _torch()
    _say("determinism / resume / subset / checkpoints")
    spec = CONFIGS["small"]
    vol = make_volume(spec, planes=6)
    planes = [oracle.reslice(s).astype(np.float32) for s in vol["stacks"]]
    obs = [_dev(p) for p in planes]
    d = Deconvolver(2, spec.n_z, spec.n_x, 0)
    for v, p in enumerate(vol["psfs"]):
        d.set_psf(v, p)
    a = d.run(obs, iters=6, layout="planes_yzx").cpu().numpy()
    b = d.run(obs, iters=6, layout="planes_yzx").cpu().numpy()
    np.testing.assert_array_equal(a, b)
    # resume: 4 + 2 iterations from the stored estimate
    e4 = d.run(obs, iters=4, layout="planes_yzx")
    r = d.run(obs, iters=2, layout="planes_yzx", init="given", est=e4.clone()).cpu().numpy()
    np.testing.assert_array_equal(a, r)
    # plane subset
    sub = [_dev(p[2:5]) for p in planes]
    s = d.run(sub, iters=6, layout="planes_yzx").cpu().numpy()
    np.testing.assert_array_equal(a[2:5], s)
    # checkpoints: slot t holds ψ^t
    ck = torch.empty((6, 6, spec.n_z, spec.n_x), dtype=torch.float32, device="cuda:0")
    c = d.run(obs, iters=6, layout="planes_yzx", checkpoints=ck).cpu().numpy()
    np.testing.assert_array_equal(a, c)
    for t in (0, 1, 5):
        et = d.run(obs, iters=t, layout="planes_yzx").cpu().numpy()
        np.testing.assert_array_equal(ck[t].cpu().numpy(), et)
    d.close()


# ---------------------------------------------------------------------------
# Paper-like workloads at reduced plane counts
# ---------------------------------------------------------------------------
def test_four_views_sequential():
    _say("4 views 0/90/180/270, 41x41, sequential, 96x96")
    rng = np.random.default_rng(14)
    psfs = [gaussian_psf(41, *s).astype(np.float32) for s in [(1.5, 8), (8, 1.5), (1.5, 8), (8, 1.5)]]
    stacks = [rng.poisson(rng.uniform(80, 400, (96, 3, 96))).astype(np.uint16) for _ in range(4)]
    got = gpu_run(stacks, psfs, 10, update="sequential")
    ref = oracle_run(stacks, psfs, 10, update="sequential")
    check(got, ref)


@pytest.mark.parametrize("name", ["mix_a", "mix_b", "mix_c"])
def test_batched_mix_volumes_sampled(name):
    _say(f"{name}: 3 planes, sequential")
    spec = CONFIGS[name]
    vol = make_volume(spec, planes=3, truth=False)
    got = gpu_run(vol["stacks"], vol["psfs"], spec.iters, update="sequential")
    ref = oracle_run(vol["stacks"], vol["psfs"], spec.iters, update="sequential", method="fft")
    check(got, ref)


@pytest.mark.parametrize("normalize", [False, True], ids=["plain", "normalised"])
def test_full_size_vol512_sampled_planes(normalize):
    """The 512³, 2-view, 31×31 workload at full size in the bench's launch
    configuration (also with the EM-normalised back-projection); 8 seeded
    planes recomputed by the oracle (planes are independent, so a sample is
    exact)."""
    _say(f"vol512 full size, sampled planes, normalize={normalize}")
    spec = CONFIGS["vol512"]
    vol = make_volume(spec, truth=False)
    got = gpu_run(vol["stacks"], vol["psfs"], spec.iters, normalize=normalize)
    rng = np.random.default_rng(512)
    ys = sorted(set([0, spec.n_planes - 1] + list(rng.choice(spec.n_planes, 6, replace=False))))
    sub = [np.ascontiguousarray(s[:, ys, :]) for s in vol["stacks"]]
    ref = oracle_run(sub, vol["psfs"], spec.iters, method="fft", normalize=normalize)
    check(got[ys], ref)


def test_planes2048_one_plane():
    """A plane of the 2048³ size class (2 views, 2048×2048, 31×31, uint16):
    rows wider than any work-group run in three strips with a 15-column halo
    under the zero boundary."""
    _say("planes2048: 1 plane of 2048x2048, 31x31, simultaneous")
    spec = CONFIGS["planes2048"]
    vol = make_volume(spec, planes=1, truth=False)
    got = gpu_run(vol["stacks"], vol["psfs"], spec.iters)
    ref = oracle_run(vol["stacks"], vol["psfs"], spec.iters, method="fft")
    check(got, ref)


def test_tuned_run_without_iterations_is_the_mean():
    """MVD_FLAG_TUNE with T = 0: no probe is made (there are no passes), so the
    run stays inside its reported workspace and returns ψ^0, the views' mean."""
    from paper_1503_07998_amd import api

    torch = _torch()
    _say("tuned run, 0 iterations")
    rng = np.random.default_rng(77)
    stacks = [rng.integers(0, 4000, (40, 6, 64)).astype(np.uint16) for _ in range(2)]
    psfs = [gaussian_psf(15, 1.5, 4.0), gaussian_psf(15, 4.0, 1.5)]
    ctx = api.mvd_create(2, 40, 64, 0)
    try:
        for v in range(2):
            api.mvd_set_psf(ctx, v, psfs[v])
        obs = [_dev(s) for s in stacks]
        est = torch.empty((6, 40, 64), dtype=torch.float32, device="cuda:0")
        run = api.make_run(6, 0, obs_dtype="u16", tune=True)
        nbytes = api.mvd_workspace_bytes(ctx, run)
        # the workspace sits at the end of its allocation: a write past it would land
        # in the guard bytes after it, which must stay untouched
        guard = 1 << 20
        buf = torch.full((nbytes + guard + 256,), 0xAB, dtype=torch.uint8, device="cuda:0")
        base = (buf.data_ptr() + 255) // 256 * 256
        run.workspace = base if nbytes else None
        run.workspace_bytes = nbytes
        api.mvd_deconvolve_planes(ctx, obs, est, run)
        torch.cuda.synchronize()
        off = base - buf.data_ptr() + nbytes
        assert bool((buf[off:off + guard] == 0xAB).all()), "the run wrote past its workspace"
        ref = oracle.deconvolve(stacks, [p.astype(np.float64) for p in psfs], 0)
        np.testing.assert_allclose(est.cpu().numpy(), ref, rtol=1e-6, atol=0)
    finally:
        api.mvd_destroy(ctx)


def test_nucleus_planewise_matches_oracle():
    """The plane-wise validation setting (one simulated nucleus, axial σ 8 px,
    lateral σ 1.5 px, 41-tap PSFs from the 3D PSFs' y-marginals, SNR 30,
    10 iterations) run on the GPU against the plane-wise oracle."""
    from oracle import full3d as F
    from synthetic import nucleus

    _say("nucleus 48x80x80, sxy 1.5, SNR 30, 10 iterations, planes layout")
    truth = nucleus((48, 80, 80), 3)
    p3 = [F.gaussian_psf3(41, 1.5, 1.5, 8.0, ky=11), F.gaussian_psf3(41, 1.5, 8.0, 1.5, ky=11)]
    rng = np.random.default_rng(5)
    obs = []
    for p in p3:
        phi = F.conv3d_fft(truth, p)
        obs.append(np.maximum(phi + rng.normal(0.0, phi.max() / 30.0, phi.shape), 0.0).astype(np.float32))
    psfs = [p.sum(axis=0).astype(np.float32) for p in p3]
    got = gpu_run(obs, psfs, 10, layout="planes_yzx")
    ref = oracle_run(obs, psfs, 10, layout="planes_yzx", method="fft")
    check(got, ref)


# ---------------------------------------------------------------------------
# Kernels of low rank (sums of rank-one terms from their SVD)
# ---------------------------------------------------------------------------
def _low_rank_psf(rng, kz, kx, r):
    """Sum of r random positive asymmetric outer products (rank r), unit sum."""
    p = sum(np.outer(rng.uniform(0.05, 1.0, kz), rng.uniform(0.05, 1.0, kx)) for _ in range(r))
    return (p / p.sum()).astype(np.float32)


LOW_RANK_CASES = [
    # (Y, Z, X, [(kz, kx, rank)], boundary, update, weights)
    (3, 37, 53, [(15, 15, 2), (21, 13, 3)], "zero", "simultaneous", None),
    (2, 70, 100, [(31, 31, 4), (31, 31, 2)], "zero", "sequential", [1.0, 0.6]),
    (3, 24, 40, [(9, 11, 3), (11, 9, 2), (7, 7, 1)], "periodic", "sequential", None),
    (2, 16, 1100, [(9, 9, 2), (9, 9, 6)], "zero", "simultaneous", None),
    (2, 13, 96, [(41, 41, 3)], "zero", "simultaneous", None),
]


@pytest.mark.parametrize("case", LOW_RANK_CASES, ids=[f"lr{i}" for i in range(len(LOW_RANK_CASES))])
def test_low_rank_psfs_match_oracle(case):
    """PSFs that are not rank one but a sum of a few outer products run as that
    many pairs of 1D passes (mvd_psf_info reports the term count) and match the
    oracle's direct K×K convolution."""
    from paper_1503_07998_amd import api

    Y, Z, X, shapes, boundary, update, weights = case
    _say(f"low rank Y={Y} Z={Z} X={X} k={shapes} {boundary} {update} w={weights}")
    rng = np.random.default_rng(zlib.crc32(repr(case).encode()))
    psfs = [_low_rank_psf(rng, kz, kx, r) for kz, kx, r in shapes]
    ctx = api.mvd_create(len(psfs), Z, X, -1)
    try:
        for v, p in enumerate(psfs):
            api.mvd_set_psf(ctx, v, p)
        for v, (_, _, r) in enumerate(shapes):
            assert api.mvd_psf_info(ctx, v) == (r, r)
    finally:
        api.mvd_destroy(ctx)
    stacks = [rng.uniform(10.0, 300.0, (Z, Y, X)).astype(np.float32) for _ in shapes]
    got = gpu_run(stacks, psfs, 5, boundary=boundary, update=update, weights=weights)
    ref = oracle_run(stacks, psfs, 5, boundary=boundary, update=update, weights=weights, method="direct")
    check(got, ref)
    # the same operator through the general K×K passes
    kxk = gpu_run(stacks, psfs, 5, boundary=boundary, update=update, weights=weights, force_2d=True)
    assert rel_err(got, kxk) <= 1e-5


@pytest.mark.parametrize("case", LOW_RANK_CASES[:4], ids=[f"lr{i}" for i in range(4)])
def test_low_rank_term_pairs_equal_single_terms(case):
    """Two terms per launch (their sum after the partial sum, in term order)
    equals one launch per term bitwise, for ranks 2 to 6 (trailing single terms
    and middle pairs included)."""
    import ctypes

    from paper_1503_07998_amd import _native as N

    Y, Z, X, shapes, boundary, update, weights = case
    _say(f"low rank pairs vs single terms Y={Y} Z={Z} X={X} k={shapes}")
    rng = np.random.default_rng(zlib.crc32(repr(case).encode()) + 1)
    psfs = [_low_rank_psf(rng, kz, kx, r) for kz, kx, r in shapes]
    stacks = [rng.uniform(10.0, 300.0, (Z, Y, X)).astype(np.float32) for _ in shapes]
    lib = N.lib()
    lib.mvd_internal_set_tune.argtypes = [ctypes.c_char_p]
    try:
        lib.mvd_internal_set_tune(b"terms=0")
        one = gpu_run(stacks, psfs, 3, boundary=boundary, update=update, weights=weights)
        lib.mvd_internal_set_tune(b"terms=1")
        two = gpu_run(stacks, psfs, 3, boundary=boundary, update=update, weights=weights)
    finally:
        lib.mvd_internal_set_tune(None)
    np.testing.assert_array_equal(two, one)


def test_low_rank_full_plane_size():
    """Two 512×512 planes of the vol512 shape with rank-two 31×31 PSFs (a main
    lobe and a weaker, wider offset lobe per view), 10 iterations, against the
    oracle (planes are independent: two planes stand for the volume)."""
    from synthetic import gaussian_psf

    _say("low rank: 2 planes of 512x512, rank-two 31x31 PSFs, 10 iterations")
    rng = np.random.default_rng(12)
    psfs = []
    for sx, sz in ((1.5, 6.0), (6.0, 1.5)):
        side = np.roll(np.roll(gaussian_psf(31, 2.0 * sx, 0.5 * sz), 3, axis=0), -2, axis=1)
        p = gaussian_psf(31, sx, sz) + 0.3 * side
        psfs.append((p / p.sum()).astype(np.float32))
    stacks = [rng.integers(80, 2000, (512, 2, 512)).astype(np.uint16) for _ in range(2)]
    got = gpu_run(stacks, psfs, 10)
    ref = oracle_run(stacks, psfs, 10, method="fft")
    check(got, ref)
