"""GPU reverse sweep (mvd_backward, mvd_backward_grads) against the FP64
oracle's adjoint: rank-one, low-rank and full-rank (K×K) PSFs, scalar and
per-pixel weights.

Bar: each gradient array within 1e-3 of the oracle's, relative to that array's
largest magnitude (float32 recomputation and float64 fixed-order reductions
against the float64 oracle); bitwise equal between two runs.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint as OA
from synthetic import CONFIGS, make_volume, random_psf

pytestmark = pytest.mark.gpu

TOL = 1e-3


def _torch():
    import torch
    return torch


def _say(msg):
    print(f"[case] {msg}", flush=True)


def gpu_forward_backward(stacks, psfs, T, gout, update="simultaneous", boundary="zero", weights=None,
                         layout="stack_zyx", weight_planes=None, plane_grads=False, force_2d=False,
                         normalize=False):
    """Forward run with checkpoints, then the reverse sweep.  weight_planes:
    per-view float32 [Y][Z][X] arrays; plane_grads: also ∂L/∂ω_v (through
    mvd_backward_grads, else mvd_backward)."""
    from paper_1503_07998_amd import api

    torch = _torch()
    dev = "cuda:0"
    obs = [torch.from_numpy(np.ascontiguousarray(s)).to(dev) for s in stacks]
    if layout == "stack_zyx":
        Z, Y, X = stacks[0].shape
    else:
        Y, Z, X = stacks[0].shape
    V = len(stacks)
    d = api.Deconvolver(V, Z, X, 0)
    for v, p in enumerate(psfs):
        d.set_psf(v, p, "flipped")
    obs_dtype = "u16" if stacks[0].dtype == np.uint16 else "f32"
    ck = torch.empty((T, Y, Z, X), dtype=torch.float32, device=dev)
    est = torch.empty((Y, Z, X), dtype=torch.float32, device=dev)
    wpl = None
    if weight_planes is not None:
        wpl = [torch.from_numpy(np.ascontiguousarray(w.astype(np.float32))).to(dev) for w in weight_planes]
    run = api.make_run(Y, T, update=update, boundary=boundary, weights=weights, checkpoints=ck.data_ptr(),
                       obs_dtype=obs_dtype, layout=layout, force_2d=force_2d, normalize=normalize,
                       weight_planes=[w.data_ptr() for w in wpl] if wpl is not None else None)
    nb = api.mvd_workspace_bytes(d.ctx, run)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
    run.workspace = (ws.data_ptr() + 255) // 256 * 256
    run.workspace_bytes = nb
    api.mvd_deconvolve_planes(d.ctx, obs, est, run)
    nb2 = api.mvd_backward_workspace_bytes(d.ctx, run)
    ws2 = torch.empty(nb2 + 256, dtype=torch.uint8, device=dev)
    run.workspace = (ws2.data_ptr() + 255) // 256 * 256
    run.workspace_bytes = nb2
    g = torch.from_numpy(np.ascontiguousarray(gout.astype(np.float32))).to(dev)
    gp = [torch.empty(p.shape, dtype=torch.float32, device=dev) for p in psfs]
    gb = [torch.empty(p.shape, dtype=torch.float32, device=dev) for p in psfs]
    gw = torch.empty(V, dtype=torch.float32, device=dev)
    gi = torch.empty((Y, Z, X), dtype=torch.float32, device=dev)
    gwp = None
    if plane_grads:
        gwp = [torch.full((Y, Z, X), -7.0, dtype=torch.float32, device=dev) for _ in range(V)]
        api.mvd_backward_grads(d.ctx, obs, g, run, gp, gb, gw, gi, gwp)
    else:
        api.mvd_backward(d.ctx, obs, g, run, gp, gb, gw, gi)
    torch.cuda.synchronize()
    out = dict(est=est.cpu().numpy(), grad_psf=[x.cpu().numpy() for x in gp],
               grad_back=[x.cpu().numpy() for x in gb], grad_weights=gw.cpu().numpy(), grad_init=gi.cpu().numpy())
    if gwp is not None:
        out["grad_weight_planes"] = [x.cpu().numpy() for x in gwp]
    d.close()
    return out


def oracle_adjoint(stacks, psfs, T, gout, update="simultaneous", boundary="zero", weights=None, method="direct",
                   normalize=False):
    phis = [oracle.reslice(s) for s in stacks]
    ps = [p.astype(np.float64) for p in psfs]
    xs = [oracle.flip(p) for p in ps]
    return OA.adjoint(phis, ps, xs, weights, T, gout, update, boundary, method=method, normalize=normalize)


def close(got, ref, name, tol=TOL):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale if scale > 0 else np.abs(got).max()
    assert err <= tol, f"{name}: max|d|/max = {err:.3e}"
    return err


CASES = [
    # (Y, Z, X, kernel shapes, T, update, boundary, weights)
    (3, 40, 48, [(9, 7), (7, 9)], 3, "simultaneous", "zero", [0.9, 0.7]),
    (2, 33, 30, [(5, 9), (9, 5)], 3, "simultaneous", "periodic", None),
    (2, 24, 40, [(7, 5), (5, 7), (3, 3)], 2, "sequential", "zero", [1.0, 0.6, 0.8]),
    (2, 17, 64, [(15, 15), (11, 11)], 2, "sequential", "periodic", None),
    # several correlation tiles along z and x' with ragged ends; 41 taps pad to 48
    (2, 37, 300, [(31, 31), (21, 41)], 2, "simultaneous", "zero", [0.8, 0.9]),
    (1, 35, 270, [(17, 33), (33, 17)], 2, "sequential", "periodic", None),
]


@pytest.fixture(params=["mfma", "valu"])
def corr_form(request):
    """Tap-gradient correlation on the matrix cores (default) or the vector ALUs."""
    import ctypes
    from paper_1503_07998_amd import _native as N

    lib = N.lib()
    lib.mvd_internal_set_tune.argtypes = [ctypes.c_char_p]
    lib.mvd_internal_set_tune(b"valu_corr=1" if request.param == "valu" else b"")
    yield request.param
    lib.mvd_internal_set_tune(None)


@pytest.mark.parametrize("case", CASES, ids=[f"a{i}" for i in range(len(CASES))])
def test_backward_matches_oracle_adjoint(case, corr_form):
    Y, Z, X, shapes, T, update, boundary, weights = case
    _say(f"backward Y={Y} Z={Z} X={X} k={shapes} T={T} {update} {boundary} w={weights} corr={corr_form}")
    rng = np.random.default_rng(Y * 1000 + Z * 10 + X)
    psfs = [random_psf(rng, kz, kx, separable=True).astype(np.float32) for kz, kx in shapes]
    stacks = [rng.uniform(20.0, 300.0, (Z, Y, X)).astype(np.float32) for _ in shapes]
    gout = rng.standard_normal((Y, Z, X))
    got = gpu_forward_backward(stacks, psfs, T, gout, update, boundary, weights)
    ref = oracle_adjoint(stacks, psfs, T, gout, update, boundary, weights)
    for v in range(len(shapes)):
        close(got["grad_psf"][v], ref["grad_psf"][v], f"grad_psf[{v}]")
        close(got["grad_back"][v], ref["grad_back"][v], f"grad_back[{v}]")
    close(got["grad_weights"], ref["grad_weights"], "grad_weights")
    close(got["grad_init"], ref["grad_psi0"], "grad_init")


PLANE_CASES = [
    # (Y, Z, X, kernel shapes, T, update, boundary, scalar weights)
    (3, 40, 48, [(9, 7), (7, 9)], 3, "simultaneous", "zero", [0.9, 0.7]),
    (2, 24, 40, [(7, 5), (5, 7), (3, 3)], 2, "sequential", "periodic", None),
    (2, 37, 130, [(31, 31), (21, 21)], 2, "sequential", "zero", [0.8, 1.0]),
    (1, 21, 33, [(5, 5), (3, 7)], 3, "simultaneous", "periodic", None),   # ragged: element-wise kernels
]


@pytest.mark.parametrize("case", PLANE_CASES, ids=[f"w{i}" for i in range(len(PLANE_CASES))])
def test_backward_with_weight_planes_matches_oracle(case):
    """Per-pixel weight planes ω_v: the reverse sweep's tap, weight and ψ^0
    gradients and ∂L/∂ω_v against the oracle's adjoint with per-pixel
    weights o_v = w_v·ω_v (∂L/∂ω_v = ∂L/∂o_v · w_v, ∂L/∂w_v = Σ ∂L/∂o_v · ω_v)."""
    Y, Z, X, shapes, T, update, boundary, weights = case
    V = len(shapes)
    _say(f"backward with weight planes Y={Y} Z={Z} X={X} k={shapes} T={T} {update} {boundary} w={weights}")
    rng = np.random.default_rng(Y * 100 + Z + X + 5)
    psfs = [random_psf(rng, kz, kx, separable=True).astype(np.float32) for kz, kx in shapes]
    stacks = [rng.uniform(20.0, 300.0, (Z, Y, X)).astype(np.float32) for _ in shapes]
    planes = [rng.uniform(0.2, 1.0, (Y, Z, X)).astype(np.float32) for _ in shapes]
    gout = rng.standard_normal((Y, Z, X))
    got = gpu_forward_backward(stacks, psfs, T, gout, update, boundary, weights, weight_planes=planes,
                               plane_grads=True)
    ws = [1.0] * V if weights is None else weights
    eff = [np.float64(ws[v]) * planes[v].astype(np.float64) for v in range(V)]
    ref = oracle_adjoint(stacks, psfs, T, gout, update, boundary, eff)
    for v in range(V):
        close(got["grad_psf"][v], ref["grad_psf"][v], f"grad_psf[{v}]")
        close(got["grad_back"][v], ref["grad_back"][v], f"grad_back[{v}]")
        close(got["grad_weight_planes"][v], ref["grad_weights"][v] * ws[v], f"grad_weight_planes[{v}]")
    gw_ref = [float(np.sum(ref["grad_weights"][v] * planes[v])) for v in range(V)]
    close(got["grad_weights"], gw_ref, "grad_weights")
    close(got["grad_init"], ref["grad_psi0"], "grad_init")
    # mvd_backward (no plane gradients) gives the same other outputs, bitwise
    alt = gpu_forward_backward(stacks, psfs, T, gout, update, boundary, weights, weight_planes=planes)
    for k in ("grad_weights", "grad_init"):
        np.testing.assert_array_equal(alt[k], got[k])
    for v in range(V):
        np.testing.assert_array_equal(alt["grad_psf"][v], got["grad_psf"][v])


def test_unit_weight_planes_equal_scalar_weights_bitwise():
    """ω_v = 1 everywhere: every gradient bitwise that of the scalar-weight run,
    and ∂L/∂ω_v sums to w_v · ∂L/∂w_v."""
    _say("backward: unit weight planes")
    rng = np.random.default_rng(123)
    shapes = [(9, 9), (7, 11)]
    psfs = [random_psf(rng, kz, kx, separable=True).astype(np.float32) for kz, kx in shapes]
    stacks = [rng.uniform(20.0, 300.0, (32, 3, 64)).astype(np.float32) for _ in shapes]
    gout = rng.standard_normal((3, 32, 64))
    ones = [np.ones((3, 32, 64), dtype=np.float32) for _ in shapes]
    for update in ("simultaneous", "sequential"):
        a = gpu_forward_backward(stacks, psfs, 2, gout, update, weights=[0.8, 0.6])
        b = gpu_forward_backward(stacks, psfs, 2, gout, update, weights=[0.8, 0.6], weight_planes=ones,
                                 plane_grads=True)
        np.testing.assert_array_equal(a["est"], b["est"])
        for k in ("grad_weights", "grad_init"):
            np.testing.assert_array_equal(a[k], b[k])
        for v in range(2):
            np.testing.assert_array_equal(a["grad_psf"][v], b["grad_psf"][v])
            np.testing.assert_array_equal(a["grad_back"][v], b["grad_back"][v])
            gwp = b["grad_weight_planes"][v].astype(np.float64)
            s, want = float(gwp.sum()), (0.8, 0.6)[v] * float(a["grad_weights"][v])
            assert abs(s - want) <= 1e-5 * float(np.abs(gwp).sum()), (update, v, s, want)


def _low_rank_psf(rng, kz, kx, r):
    """Sum of r random positive asymmetric outer products (rank r), unit sum."""
    p = sum(np.outer(rng.uniform(0.05, 1.0, kz), rng.uniform(0.05, 1.0, kx)) for _ in range(r))
    return (p / p.sum()).astype(np.float32)


LOW_RANK_CASES = [
    # (Y, Z, X, [(kz, kx, rank)], T, update, boundary, weights); rank 1 = separable
    (2, 37, 53, [(15, 15, 2), (13, 21, 3)], 3, "simultaneous", "zero", [0.9, 0.7]),
    (2, 30, 44, [(9, 11, 3), (11, 9, 1), (7, 7, 2)], 2, "sequential", "periodic", None),
    (1, 45, 70, [(31, 31, 4), (21, 21, 1)], 2, "sequential", "zero", [1.0, 0.8]),
    (2, 21, 33, [(9, 9, 6)], 2, "simultaneous", "zero", None),     # ragged, six terms
]


@pytest.mark.parametrize("case", LOW_RANK_CASES, ids=[f"lr{i}" for i in range(len(LOW_RANK_CASES))])
def test_backward_low_rank_psfs_match_oracle(case):
    """PSFs that are sums of a few rank-one terms: the reverse sweep sums the
    terms pass by pass and finishes the ratio and b̄ pointwise; the tap
    gradients cover the whole K×K kernel.  Against the oracle's K×K adjoint."""
    from paper_1503_07998_amd import api

    Y, Z, X, shapes, T, update, boundary, weights = case
    _say(f"backward low rank Y={Y} Z={Z} X={X} k={shapes} T={T} {update} {boundary} w={weights}")
    rng = np.random.default_rng(Y * 7 + Z * 3 + X)
    psfs = [_low_rank_psf(rng, kz, kx, r) for kz, kx, r in shapes]
    ctx = api.mvd_create(len(psfs), Z, X, -1)
    try:
        for v, p in enumerate(psfs):
            api.mvd_set_psf(ctx, v, p)
        for v, (_, _, r) in enumerate(shapes):
            assert api.mvd_psf_info(ctx, v) == (r, r)
    finally:
        api.mvd_destroy(ctx)
    stacks = [rng.uniform(20.0, 300.0, (Z, Y, X)).astype(np.float32) for _ in shapes]
    gout = rng.standard_normal((Y, Z, X))
    got = gpu_forward_backward(stacks, psfs, T, gout, update, boundary, weights)
    ref = oracle_adjoint(stacks, psfs, T, gout, update, boundary, weights)
    for v in range(len(shapes)):
        close(got["grad_psf"][v], ref["grad_psf"][v], f"grad_psf[{v}]")
        close(got["grad_back"][v], ref["grad_back"][v], f"grad_back[{v}]")
    close(got["grad_weights"], ref["grad_weights"], "grad_weights")
    close(got["grad_init"], ref["grad_psi0"], "grad_init")


KXK_CASES = [
    # (Y, Z, X, [(kz, kx, full)], T, update, boundary, weights, force_2d); full: a full-rank kernel
    (2, 30, 40, [(9, 9, True), (7, 11, True)], 2, "simultaneous", "zero", [0.9, 0.8], False),
    (2, 24, 50, [(15, 15, True), (5, 5, False)], 2, "sequential", "periodic", None, False),
    (1, 33, 70, [(31, 31, True), (21, 21, True)], 2, "simultaneous", "zero", None, False),
    (2, 26, 45, [(9, 7, False), (7, 9, False)], 3, "sequential", "zero", [1.0, 0.7], True),   # K×K forced
]


@pytest.mark.parametrize("case", KXK_CASES, ids=[f"kxk{i}" for i in range(len(KXK_CASES))])
def test_backward_kxk_psfs_match_oracle(case):
    """Full-rank PSFs (the K×K passes, which store the convolution and finish
    the ratio, b̄ and ψ̄ pointwise) and runs forced onto the K×K passes,
    against the oracle's adjoint."""
    from paper_1503_07998_amd import api

    Y, Z, X, shapes, T, update, boundary, weights, force_2d = case
    _say(f"backward K×K Y={Y} Z={Z} X={X} k={shapes} T={T} {update} {boundary} w={weights} force_2d={force_2d}")
    rng = np.random.default_rng(Y * 11 + Z * 5 + X)
    psfs = [random_psf(rng, kz, kx, separable=not full).astype(np.float32) for kz, kx, full in shapes]
    ctx = api.mvd_create(len(psfs), Z, X, -1)
    try:
        for v, p in enumerate(psfs):
            api.mvd_set_psf(ctx, v, p)
        for v, (_, _, full) in enumerate(shapes):
            assert api.mvd_psf_info(ctx, v) == ((0, 0) if full else (1, 1))
    finally:
        api.mvd_destroy(ctx)
    stacks = [rng.uniform(20.0, 300.0, (Z, Y, X)).astype(np.float32) for _ in shapes]
    gout = rng.standard_normal((Y, Z, X))
    got = gpu_forward_backward(stacks, psfs, T, gout, update, boundary, weights, force_2d=force_2d)
    ref = oracle_adjoint(stacks, psfs, T, gout, update, boundary, weights)
    for v in range(len(shapes)):
        close(got["grad_psf"][v], ref["grad_psf"][v], f"grad_psf[{v}]")
        close(got["grad_back"][v], ref["grad_back"][v], f"grad_back[{v}]")
    close(got["grad_weights"], ref["grad_weights"], "grad_weights")
    close(got["grad_init"], ref["grad_psi0"], "grad_init")


NORM_CASES = [
    # (Y, Z, X, [(kz, kx, rank: 1 separable, 0 full, r low)], T, update, boundary, weights, weight planes)
    (2, 30, 44, [(9, 7, 1), (7, 11, 1)], 3, "simultaneous", "zero", [0.9, 0.8], False),
    (2, 26, 37, [(11, 11, 1), (5, 9, 1), (7, 7, 1)], 2, "sequential", "zero", None, False),
    (2, 24, 48, [(9, 13, 1), (7, 7, 1)], 2, "simultaneous", "periodic", None, False),
    (1, 40, 64, [(31, 31, 1), (21, 21, 1)], 2, "sequential", "zero", [1.0, 0.7], True),
    # back-projectors that are not rank one (the general update and sensitivity planes)
    (2, 28, 40, [(9, 9, 3), (7, 7, 0)], 2, "simultaneous", "zero", [0.9, 0.8], False),
    (2, 25, 36, [(9, 9, 0), (7, 9, 2)], 2, "sequential", "zero", None, True),
]


@pytest.mark.parametrize("case", NORM_CASES, ids=[f"n{i}" for i in range(len(NORM_CASES))])
def test_backward_normalised_matches_oracle(case):
    """EM-normalised back-projection: the chain rule through q / s_v and
    through s_v = 1 ⊛ X_v (whose tap gradient is s̄'s correlation with a plane
    of ones), against the oracle's normalised adjoint; with weight planes too."""
    Y, Z, X, shapes, T, update, boundary, weights, with_planes = case
    V = len(shapes)
    _say(f"backward normalised Y={Y} Z={Z} X={X} k={shapes} T={T} {update} {boundary} w={weights} "
         f"planes={with_planes}")
    rng = np.random.default_rng(Y * 13 + Z * 7 + X)
    psfs = [(random_psf(rng, kz, kx, separable=(r == 1)) if r <= 1 else _low_rank_psf(rng, kz, kx, r))
            .astype(np.float32) for kz, kx, r in shapes]
    stacks = [rng.uniform(20.0, 300.0, (Z, Y, X)).astype(np.float32) for _ in shapes]
    gout = rng.standard_normal((Y, Z, X))
    planes = [rng.uniform(0.2, 1.0, (Y, Z, X)).astype(np.float32) for _ in shapes] if with_planes else None
    got = gpu_forward_backward(stacks, psfs, T, gout, update, boundary, weights, weight_planes=planes,
                               normalize=True)
    ws = [1.0] * V if weights is None else weights
    eff = [np.float64(ws[v]) * planes[v].astype(np.float64) for v in range(V)] if with_planes else weights
    ref = oracle_adjoint(stacks, psfs, T, gout, update, boundary, eff, normalize=True)
    for v in range(V):
        close(got["grad_psf"][v], ref["grad_psf"][v], f"grad_psf[{v}]")
        close(got["grad_back"][v], ref["grad_back"][v], f"grad_back[{v}]")
    if with_planes:
        close(got["grad_weights"], [float(np.sum(ref["grad_weights"][v] * planes[v])) for v in range(V)],
              "grad_weights")
    else:
        close(got["grad_weights"], ref["grad_weights"], "grad_weights")
    close(got["grad_init"], ref["grad_psi0"], "grad_init")


def test_backward_is_deterministic():
    _say("backward determinism")
    rng = np.random.default_rng(77)
    psfs = [random_psf(rng, 9, 9, separable=True).astype(np.float32) for _ in range(2)]
    stacks = [rng.uniform(20.0, 300.0, (64, 4, 64)).astype(np.float32) for _ in range(2)]
    gout = rng.standard_normal((4, 64, 64))
    a = gpu_forward_backward(stacks, psfs, 3, gout)
    b = gpu_forward_backward(stacks, psfs, 3, gout)
    for k in ("grad_weights", "grad_init"):
        np.testing.assert_array_equal(a[k], b[k])
    for v in range(2):
        np.testing.assert_array_equal(a["grad_psf"][v], b["grad_psf"][v])
        np.testing.assert_array_equal(a["grad_back"][v], b["grad_back"][v])


def test_correlation_forms_agree():
    """Matrix-core and vector-ALU correlations give the same tap gradients up
    to float32 summation order."""
    import ctypes
    from paper_1503_07998_amd import _native as N

    _say("correlation forms agree, 4 planes of 48x200, 31x31 and 41x41")
    rng = np.random.default_rng(91)
    psfs = [random_psf(rng, 31, 31, separable=True).astype(np.float32),
            random_psf(rng, 41, 41, separable=True).astype(np.float32)]
    stacks = [rng.uniform(20.0, 300.0, (48, 4, 200)).astype(np.float32) for _ in range(2)]
    gout = rng.standard_normal((4, 48, 200))
    lib = N.lib()
    lib.mvd_internal_set_tune.argtypes = [ctypes.c_char_p]
    try:
        lib.mvd_internal_set_tune(b"")
        a = gpu_forward_backward(stacks, psfs, 2, gout)
        lib.mvd_internal_set_tune(b"valu_corr=1")
        b = gpu_forward_backward(stacks, psfs, 2, gout)
    finally:
        lib.mvd_internal_set_tune(None)
    for v in range(2):
        close(a["grad_psf"][v], b["grad_psf"][v], f"grad_psf[{v}]", tol=1e-5)
        close(a["grad_back"][v], b["grad_back"][v], f"grad_back[{v}]", tol=1e-5)
    np.testing.assert_array_equal(a["grad_init"], b["grad_init"])


def test_grad256_planes_match_oracle():
    """The differentiation workload (2 views, 256×256 planes, 31×31 PSFs,
    5 iterations, MSE to the truth) on 2 planes at full plane size."""
    _say("grad256 workload, 2 planes")
    spec = CONFIGS["grad256"]
    vol = make_volume(spec, planes=2)
    truth = np.ascontiguousarray(np.transpose(vol["truth"], (1, 0, 2))).astype(np.float64)
    # forward on the GPU to get ψ^T, then ∂L/∂ψ^T of the MSE
    from paper_1503_07998_amd import deconvolve
    torch = _torch()
    est = deconvolve([torch.from_numpy(s).to("cuda:0") for s in vol["stacks"]], vol["psfs"],
                     iters=spec.iters).cpu().numpy().astype(np.float64)
    _, gout = OA.mse_loss_and_grad(est, truth)
    got = gpu_forward_backward(vol["stacks"], vol["psfs"], spec.iters, gout, weights=[0.9, 0.8])
    ref = oracle_adjoint(vol["stacks"], vol["psfs"], spec.iters, gout, weights=[0.9, 0.8], method="fft")
    for v in range(2):
        close(got["grad_psf"][v], ref["grad_psf"][v], f"grad_psf[{v}]")
        close(got["grad_back"][v], ref["grad_back"][v], f"grad_back[{v}]")
    close(got["grad_weights"], ref["grad_weights"], "grad_weights")


def test_autograd_sigma_gradients():
    """σ and weight gradients through torch.autograd vs the oracle's chain."""
    from paper_1503_07998_amd.autograd import PlanewiseRL

    torch = _torch()
    _say("autograd sigma gradients")
    rng = np.random.default_rng(9)
    Y, Z, X, k, T = 2, 40, 36, 11, 3
    truth = 100.0 + 600.0 * (rng.random((Y, Z, X)) > 0.95)
    data_sig = [(1.5, 3.0), (3.0, 1.5)]
    phis = [oracle.conv2d(truth, OA.gaussian_taps(k, *s)[0]) + rng.uniform(0, 2, truth.shape) for s in data_sig]
    stacks = [np.ascontiguousarray(np.transpose(p, (1, 0, 2))).astype(np.float32) for p in phis]
    sig = [(1.7, 3.3), (3.2, 1.6)]
    ws = [0.9, 0.8]
    prob = PlanewiseRL([torch.from_numpy(s).to("cuda:0") for s in stacks], k, T)
    sigma = torch.tensor(sig, dtype=torch.float64, requires_grad=True)
    w = torch.tensor(ws, dtype=torch.float64, requires_grad=True)
    psi = prob(sigma, w)
    loss = ((psi.double() - torch.from_numpy(truth).to("cuda:0")) ** 2).mean()
    loss.backward()
    phis32 = [oracle.reslice(s) for s in stacks]
    ref_loss, ref_gs, ref_gw = OA.sigma_gradients(phis32, sig, ws, T, truth, k)
    assert abs(loss.item() - ref_loss) <= 1e-4 * ref_loss
    close(sigma.grad.numpy(), ref_gs, "dL/dsigma")
    close(w.grad.numpy(), ref_gw, "dL/dw")
    prob.dec.close()


def test_autograd_backward_uses_its_own_forward_sigma():
    """forward(σ1), forward(σ2), then backward of the first: the reverse sweep
    must recompute with σ1's taps (the context holds σ2's after the second call)."""
    from paper_1503_07998_amd.autograd import PlanewiseRL

    torch = _torch()
    _say("autograd: backward after an interleaved forward")
    rng = np.random.default_rng(19)
    Y, Z, X, k, T = 2, 32, 40, 11, 3
    truth = 100.0 + 600.0 * (rng.random((Y, Z, X)) > 0.95)
    data_sig = [(1.5, 3.0), (3.0, 1.5)]
    phis = [oracle.conv2d(truth, OA.gaussian_taps(k, *s)[0]) + rng.uniform(0, 2, truth.shape) for s in data_sig]
    stacks = [np.ascontiguousarray(np.transpose(p, (1, 0, 2))).astype(np.float32) for p in phis]
    sig1, sig2 = [(1.7, 3.3), (3.2, 1.6)], [(2.4, 2.1), (1.9, 2.8)]
    ws = [0.9, 0.8]
    prob = PlanewiseRL([torch.from_numpy(s).to("cuda:0") for s in stacks], k, T)
    s1 = torch.tensor(sig1, dtype=torch.float64, requires_grad=True)
    w1 = torch.tensor(ws, dtype=torch.float64, requires_grad=True)
    psi1 = prob(s1, w1)
    s2 = torch.tensor(sig2, dtype=torch.float64, requires_grad=True)
    _ = prob(s2, torch.tensor(ws, dtype=torch.float64))
    loss = ((psi1.double() - torch.from_numpy(truth).to("cuda:0")) ** 2).mean()
    loss.backward()
    phis32 = [oracle.reslice(s) for s in stacks]
    ref_loss, ref_gs, ref_gw = OA.sigma_gradients(phis32, sig1, ws, T, truth, k)
    assert abs(loss.item() - ref_loss) <= 1e-4 * ref_loss
    close(s1.grad.numpy(), ref_gs, "dL/dsigma (first forward)")
    close(w1.grad.numpy(), ref_gw, "dL/dw (first forward)")
    prob.dec.close()


@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
def test_autograd_taps_weight_planes_normalised(update):
    """torch autograd through the library with PSF taps given directly (one
    low-rank and one full-rank kernel), per-pixel weight planes and the
    EM-normalised back-projection: ∂L/∂taps (= ∂L/∂P + flip(∂L/∂X)), ∂L/∂w and
    ∂L/∂ω against the oracle's adjoint."""
    from paper_1503_07998_amd.autograd import PlanewiseRL, mv_deconvolve_taps

    torch = _torch()
    _say(f"autograd: taps, weight planes, normalised, {update}")
    rng = np.random.default_rng(29)
    Y, Z, X, k, T = 2, 30, 38, 9, 2
    psfs = [_low_rank_psf(rng, k, k, 2), random_psf(rng, k, k).astype(np.float32)]
    stacks = [rng.uniform(20.0, 300.0, (Z, Y, X)).astype(np.float32) for _ in range(2)]
    om = np.stack([rng.uniform(0.2, 1.0, (Y, Z, X)) for _ in range(2)]).astype(np.float32)
    ws = [0.9, 0.7]
    gout = rng.standard_normal((Y, Z, X))
    prob = PlanewiseRL([torch.from_numpy(s).to("cuda:0") for s in stacks], k, T, update=update, normalize=True)
    taps = torch.tensor(np.stack(psfs), dtype=torch.float64, requires_grad=True)
    w = torch.tensor(ws, dtype=torch.float64, requires_grad=True)
    planes = torch.from_numpy(om).to("cuda:0").requires_grad_(True)
    psi = mv_deconvolve_taps(taps, w, prob, planes)
    (psi.double() * torch.from_numpy(gout).to("cuda:0")).sum().backward()
    eff = [np.float64(ws[v]) * om[v].astype(np.float64) for v in range(2)]
    ref = oracle_adjoint(stacks, psfs, T, gout, update, "zero", eff, normalize=True)
    for v in range(2):
        close(taps.grad[v].numpy(), ref["grad_psf"][v] + oracle.flip(ref["grad_back"][v]), f"dL/dtaps[{v}]")
        close(planes.grad[v].cpu().numpy(), ref["grad_weights"][v] * ws[v], f"dL/domega[{v}]")
    close(w.grad.numpy(), [float(np.sum(ref["grad_weights"][v] * om[v])) for v in range(2)], "dL/dw")
    prob.dec.close()
