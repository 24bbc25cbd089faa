"""Graph capture and the batched form against the plain path.

A captured run is replayed several times with the program's own eager work
and synchronisations between the replays; every replay must equal the eager
result bitwise.  The batched form (one graph, one branch per volume) must
equal the plain per-volume runs, and both stay within 1e-4 of the oracle.
"""
import numpy as np
import pytest

import oracle
from synthetic import CONFIGS, make_volume

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _setup(spec, planes, dev="cuda:0"):
    from paper_1503_07998_amd import api

    torch = _torch()
    vol = make_volume(spec, planes=planes, truth=False)
    obs = [torch.from_numpy(s).to(dev) for s in vol["stacks"]]
    d = api.Deconvolver(spec.n_views, spec.n_z, spec.n_x, 0)
    for v, p in enumerate(vol["psfs"]):
        d.set_psf(v, p)
    est = torch.empty((planes, spec.n_z, spec.n_x), dtype=torch.float32, device=dev)
    run = api.make_run(planes, spec.iters, update=spec.update, boundary=spec.boundary,
                       obs_dtype=spec.obs_dtype, layout="stack_zyx")
    nb = api.mvd_workspace_bytes(d.ctx, run)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
    run.workspace = (ws.data_ptr() + 255) // 256 * 256
    run.workspace_bytes = nb
    return dict(vol=vol, obs=obs, dec=d, est=est, run=run, ws=ws)


def test_graph_replays_match_eager():
    from paper_1503_07998_amd import api

    torch = _torch()
    _say("graph capture vs eager, 4 replays with eager work between")
    st = _setup(CONFIGS["small"], 6)
    d, obs, est, run = st["dec"], st["obs"], st["est"], st["run"]
    api.mvd_deconvolve_planes(d.ctx, obs, est, run)
    torch.cuda.synchronize()
    eager = est.cpu().numpy().copy()
    run.flags |= 0x4   # MVD_FLAG_GRAPH
    scratch = torch.zeros(1 << 20, device="cuda:0")
    for rep in range(4):
        est.fill_(-1.0)
        api.mvd_deconvolve_planes(d.ctx, obs, est, run)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(est.cpu().numpy(), eager)
        scratch.add_(1.0)              # unrelated eager work between replays
        _ = scratch.sum().item()
    d.close()


def test_batch_matches_plain_runs():
    from paper_1503_07998_amd import api

    torch = _torch()
    _say("batched mix (3 planes per volume) vs plain")
    specs = [CONFIGS["mix_a"], CONFIGS["mix_b"], CONFIGS["mix_c"]]
    setups = [_setup(sp, 3) for sp in specs]
    plain = []
    for st in setups:
        api.mvd_deconvolve_planes(st["dec"].ctx, st["obs"], st["est"], st["run"])
        torch.cuda.synchronize()
        plain.append(st["est"].cpu().numpy().copy())
    entries = [(st["dec"].ctx, st["obs"], st["est"], st["run"]) for st in setups]
    for tune in (False, True):
        b = api.Batch(entries, tune=tune)
        for rep in range(3):
            for st in setups:
                st["est"].fill_(-1.0)
            b.launch()
            torch.cuda.synchronize()
            for st, ref in zip(setups, plain):
                got = st["est"].cpu().numpy()
                err = np.abs(got - ref).max() / np.abs(ref).max()
                assert err <= 1e-6, f"batched vs plain: {err:.3e} (tune={tune})"
        b.close()
    # the batch and the plain path against the oracle on one volume
    st, sp = setups[0], specs[0]
    ref = oracle.deconvolve(st["vol"]["stacks"], [p.astype(np.float64) for p in st["vol"]["psfs"]], sp.iters,
                            update=sp.update, method="fft")
    assert np.abs(plain[0] - ref).max() / np.abs(ref).max() <= 1e-4
    for st in setups:
        st["dec"].close()


def test_batch_run_one_shot_and_validation():
    from paper_1503_07998_amd import _native as N
    from paper_1503_07998_amd import api

    torch = _torch()
    _say("mvd_batch_run and item validation")
    st = _setup(CONFIGS["small"], 2)
    api.mvd_batch_run([(st["dec"].ctx, st["obs"], st["est"], st["run"])])
    got = st["est"].cpu().numpy().copy()
    api.mvd_deconvolve_planes(st["dec"].ctx, st["obs"], st["est"], st["run"])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got, st["est"].cpu().numpy())
    bad = api.make_run(2, 10)     # no workspace
    with pytest.raises(N.MvdError) as e:
        api.mvd_batch_create([(st["dec"].ctx, st["obs"], st["est"], bad)])
    assert e.value.status == N.MVD_ERR_WORKSPACE
    st["dec"].close()


def test_tuned_run_matches_plain():
    """MVD_FLAG_TUNE times launch-shape candidates on the first call of a shape
    and caches the choice; results equal the untuned run up to float32
    rounding (several views' factors may be applied in one launch)."""
    from paper_1503_07998_amd import api

    torch = _torch()
    _say("tuned run vs plain (mix_b shape, 3 planes), then cached")
    st = _setup(CONFIGS["mix_b"], 3)
    d, obs, est, run = st["dec"], st["obs"], st["est"], st["run"]
    api.mvd_deconvolve_planes(d.ctx, obs, est, run)
    torch.cuda.synchronize()
    plain = est.cpu().numpy().copy()
    run.flags |= 0x8   # MVD_FLAG_TUNE
    for rep in range(2):
        est.fill_(-1.0)
        api.mvd_deconvolve_planes(d.ctx, obs, est, run)
        torch.cuda.synchronize()
        got = est.cpu().numpy()
        err = np.abs(got - plain).max() / np.abs(plain).max()
        assert err <= 1e-6, f"tuned vs plain: {err:.3e} (call {rep})"
    run.flags |= 0x4   # tuned and captured
    for rep in range(2):
        est.fill_(-1.0)
        api.mvd_deconvolve_planes(d.ctx, obs, est, run)
        torch.cuda.synchronize()
        err = np.abs(est.cpu().numpy() - plain).max() / np.abs(plain).max()
        assert err <= 1e-6, f"tuned graph vs plain: {err:.3e}"
    d.close()


def _planes_case(nz, nx, ny, views, k, iters, update, seed, *, dtype="f32", layout="stack_zyx", boundary="zero",
                 init="mean", weights=None, periodic_ok=True):
    """A seeded volume with its own context, workspace and run (not from CONFIGS)."""
    from paper_1503_07998_amd import api
    from synthetic import gaussian_psf, random_psf

    torch = _torch()
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx) if layout == "stack_zyx" else (ny, nz, nx)
    if dtype == "u16":
        stacks = [rng.integers(50, 3000, shape).astype(np.uint16) for _ in range(views)]
    else:
        stacks = [rng.uniform(50.0, 3000.0, shape).astype(np.float32) for _ in range(views)]
    psfs = [random_psf(rng, k, k, separable=True) if v % 2 else gaussian_psf(k, 1.2 + 0.3 * v, 2.5) for v in range(views)]
    d = api.Deconvolver(views, nz, nx, 0)
    for v, p in enumerate(psfs):
        d.set_psf(v, p)
    obs = [torch.from_numpy(s).to("cuda:0") for s in stacks]
    est = torch.empty((ny, nz, nx), dtype=torch.float32, device="cuda:0")
    run = api.make_run(ny, iters, update=update, boundary=boundary, init=init, init_const=150.0,
                       obs_dtype=dtype, layout=layout, weights=weights)
    nb = api.mvd_workspace_bytes(d.ctx, run)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda:0")
    run.workspace = (ws.data_ptr() + 255) // 256 * 256
    run.workspace_bytes = nb
    given = torch.from_numpy(rng.uniform(80.0, 200.0, (ny, nz, nx)).astype(np.float32)).to("cuda:0")
    return dict(obs=obs, dec=d, est=est, run=run, ws=ws, init=init, given=given,
                stacks=stacks, psfs=psfs, update=update, iters=iters)


def _reset(st):
    if st["init"] == "given":
        st["est"].copy_(st["given"])
    else:
        st["est"].fill_(-1.0)


def _plain(st):
    from paper_1503_07998_amd import api

    torch = _torch()
    _reset(st)
    api.mvd_deconvolve_planes(st["dec"].ctx, st["obs"], st["est"], st["run"])
    torch.cuda.synchronize()
    return st["est"].cpu().numpy().copy()


def _persistent_cases():
    return [
        # the three mix shapes, fewer planes
        dict(nz=256, nx=384, ny=3, views=2, k=21, iters=3, update="sequential", seed=1),
        dict(nz=128, nx=768, ny=2, views=3, k=31, iters=2, update="sequential", seed=2),
        dict(nz=100, nx=1000, ny=2, views=4, k=41, iters=2, update="sequential", seed=3),
        # simultaneous, two views in one forward pass, uint16 stacks
        dict(nz=64, nx=96, ny=5, views=2, k=31, iters=3, update="simultaneous", seed=4, dtype="u16"),
        # simultaneous, three views (views in pairs: (0, 1), (2)), planes layout, weights
        dict(nz=40, nx=64, ny=4, views=3, k=15, iters=3, update="simultaneous", seed=5, layout="planes_yzx",
             weights=[1.0, 0.7, 0.5]),
        # periodic boundary (column strips with wrapped halos), small kernels, constant ψ^0
        dict(nz=24, nx=48, ny=3, views=1, k=3, iters=4, update="sequential", seed=6, boundary="periodic",
             init="const"),
        dict(nz=33, nx=40, ny=3, views=2, k=7, iters=2, update="simultaneous", seed=7, init="given"),
    ]


def test_persistent_batch_equals_plain_bitwise():
    """Every volume of one persistent launch equals its plain run bitwise, on
    three launches in a row (the queue and the per-plane counters reset
    themselves at the end of each launch)."""
    from paper_1503_07998_amd import api

    torch = _torch()
    _say("persistent batch of 7 volumes vs plain runs, 3 launches")
    setups = [_planes_case(**c) for c in _persistent_cases()]
    plain = [_plain(st) for st in setups]
    entries = [(st["dec"].ctx, st["obs"], st["est"], st["run"]) for st in setups]
    b = api.Batch(entries)
    info = b.info()
    assert info["persistent"], info
    assert info["work_groups"] >= 256
    for rep in range(3):
        for st in setups:
            _reset(st)
        b.launch()
        b.wait()
        for i, (st, ref) in enumerate(zip(setups, plain)):
            np.testing.assert_array_equal(st["est"].cpu().numpy(), ref, err_msg=f"volume {i}, launch {rep}")
    b.close()
    # the plain path itself against the oracle (one simultaneous and one sequential volume)
    for i in (3, 0):
        st = setups[i]
        ref = oracle.deconvolve(st["stacks"], [np.asarray(p, dtype=np.float64) for p in st["psfs"]], st["iters"],
                                update=st["update"], method="fft")
        assert np.abs(plain[i] - ref).max() / np.abs(ref).max() <= 1e-4
    for st in setups:
        st["dec"].close()


def test_persistent_batch_windows_and_graph_fallback():
    """Windows of planes change only the order of the work, not the results;
    an item the persistent kernel does not take (rows not a multiple of 8
    columns) makes the batch a graph, with the same results."""
    from paper_1503_07998_amd import _native as N
    from paper_1503_07998_amd import api
    import ctypes

    torch = _torch()
    _say("persistent batch with 2-plane windows; graph fallback")
    cases = _persistent_cases()[:4]
    setups = [_planes_case(**c) for c in cases]
    plain = [_plain(st) for st in setups]
    lib = N.lib()
    lib.mvd_internal_set_tune.argtypes = [ctypes.c_char_p]
    try:
        lib.mvd_internal_set_tune(b"pq_window=2")
        b = api.Batch([(st["dec"].ctx, st["obs"], st["est"], st["run"]) for st in setups])
    finally:
        lib.mvd_internal_set_tune(None)
    assert b.info()["persistent"]
    for st in setups:
        _reset(st)
    b.launch()
    b.wait()
    for st, ref in zip(setups, plain):
        np.testing.assert_array_equal(st["est"].cpu().numpy(), ref)
    b.close()
    odd = _planes_case(nz=20, nx=37, ny=3, views=2, k=5, iters=2, update="simultaneous", seed=9)
    ref = _plain(odd)
    b = api.Batch([(odd["dec"].ctx, odd["obs"], odd["est"], odd["run"]),
                   (setups[0]["dec"].ctx, setups[0]["obs"], setups[0]["est"], setups[0]["run"])])
    assert not b.info()["persistent"]
    _reset(odd)
    _reset(setups[0])
    b.launch()
    b.wait()
    np.testing.assert_array_equal(odd["est"].cpu().numpy(), ref)
    np.testing.assert_array_equal(setups[0]["est"].cpu().numpy(), plain[0])
    b.close()
    for st in setups + [odd]:
        st["dec"].close()


def test_persistent_give_up_is_reported():
    """A raised give-up flag (as a wait that exceeded its spin limit would
    raise it) makes every work-group skip the rest and end; the host gets
    MVD_ERR_LAUNCH, and the next launch runs normally.  A spin limit of one
    poll either gives up (reported) or, where no wait was needed, leaves the
    result exact: never a silent wrong result."""
    from paper_1503_07998_amd import _native as N
    from paper_1503_07998_amd import api
    import ctypes

    torch = _torch()
    _say("persistent batch: give-up flag reported, then a normal launch")
    st = _planes_case(nz=512, nx=512, ny=2, views=2, k=31, iters=2, update="simultaneous", seed=11)
    ref = _plain(st)
    b = api.Batch([(st["dec"].ctx, st["obs"], st["est"], st["run"])])
    lib = N.lib()
    lib.mvd_internal_batch_raise_giveup.argtypes = [ctypes.c_void_p]
    assert lib.mvd_internal_batch_raise_giveup(b.handle) == 0
    _reset(st)
    b.launch()
    with pytest.raises(N.MvdError) as e:
        b.wait()
    assert e.value.status == N.MVD_ERR_LAUNCH
    _reset(st)
    b.launch()
    b.wait()
    np.testing.assert_array_equal(st["est"].cpu().numpy(), ref)
    lib.mvd_internal_set_pq_spin.argtypes = [ctypes.c_uint]
    try:
        lib.mvd_internal_set_pq_spin(1)
        _reset(st)
        b.launch()
        try:
            b.wait()
            np.testing.assert_array_equal(st["est"].cpu().numpy(), ref)
        except N.MvdError as err:
            assert err.status == N.MVD_ERR_LAUNCH
    finally:
        lib.mvd_internal_set_pq_spin(0)
    _reset(st)
    b.launch()
    b.wait()
    np.testing.assert_array_equal(st["est"].cpu().numpy(), ref)
    b.close()
    st["dec"].close()


def test_batch_of_composed_variants_equals_plain():
    """Items that combine the variants (normalised back-projection, per-pixel
    weight planes, a low-rank and a full-rank PSF, forced K×K passes) take the
    graph form and equal their plain runs bitwise."""
    from paper_1503_07998_amd import api
    from synthetic import random_psf

    torch = _torch()
    _say("batch of composed variants")
    rng = np.random.default_rng(61)

    def low_rank(k, r):
        p = sum(np.outer(rng.uniform(0.05, 1.0, k), rng.uniform(0.05, 1.0, k)) for _ in range(r))
        return (p / p.sum()).astype(np.float32)

    specs = [
        # (nz, ny, nx, psfs, update, kwargs)
        (30, 3, 40, [low_rank(9, 3), random_psf(rng, 7, 7).astype(np.float32)], "simultaneous",
         dict(normalize=True)),
        (26, 2, 48, [random_psf(rng, 9, 9, separable=True).astype(np.float32), low_rank(7, 2)], "sequential",
         dict(normalize=True, planes=True)),
        (22, 2, 36, [random_psf(rng, 5, 7, separable=True).astype(np.float32)] * 2, "sequential",
         dict(planes=True, force_2d=True)),
    ]
    setups = []
    for nz, ny, nx, psfs, update, kw in specs:
        d = api.Deconvolver(len(psfs), nz, nx, 0)
        for v, p in enumerate(psfs):
            d.set_psf(v, p)
        obs = [torch.from_numpy(rng.uniform(20.0, 400.0, (nz, ny, nx)).astype(np.float32)).to("cuda:0")
               for _ in psfs]
        planes = ([torch.from_numpy(rng.uniform(0.2, 1.0, (ny, nz, nx)).astype(np.float32)).to("cuda:0")
                   for _ in psfs] if kw.get("planes") else None)
        est = torch.empty((ny, nz, nx), dtype=torch.float32, device="cuda:0")
        run = api.make_run(ny, 3, update=update, weights=[0.9] * len(psfs), normalize=kw.get("normalize", False),
                           force_2d=kw.get("force_2d", False), weight_planes=planes)
        nb = api.mvd_workspace_bytes(d.ctx, run)
        ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda:0")
        run.workspace = (ws.data_ptr() + 255) // 256 * 256
        run.workspace_bytes = nb
        setups.append(dict(dec=d, obs=obs, est=est, run=run, ws=ws, planes=planes, init="mean"))
    plain = [_plain(st) for st in setups]
    b = api.Batch([(st["dec"].ctx, st["obs"], st["est"], st["run"]) for st in setups])
    assert not b.info()["persistent"]
    for st in setups:
        _reset(st)
    b.launch()
    b.wait()
    for st, ref in zip(setups, plain):
        got = st["est"].cpu().numpy()
        assert np.all(np.isfinite(got))
        np.testing.assert_array_equal(got, ref)
    b.close()
    for st in setups:
        st["dec"].close()


def test_tuned_batch_keeps_one_form_and_matches_plain():
    """MVD_BATCH_TUNE on items the persistent form takes: both forms are built
    and timed and one is kept; its launches agree with the plain runs (tuned
    launch shapes change summation orders only) and repeat bitwise; a given
    ψ^0 keeps the persistent form without timing."""
    from paper_1503_07998_amd import api

    _say("tuned batch: form choice")
    cases = _persistent_cases()[:2]
    setups = [_planes_case(**c) for c in cases]
    plain = [_plain(st) for st in setups]
    b = api.Batch([(st["dec"].ctx, st["obs"], st["est"], st["run"]) for st in setups], tune=True)
    form = b.info()["persistent"]
    t_pq, t_graph = b.form_times()
    assert t_pq > 0 and t_graph > 0 and form == (t_pq <= t_graph)
    outs = []
    for _ in range(2):
        for st in setups:
            _reset(st)
        b.launch()
        b.wait()
        outs.append([st["est"].cpu().numpy() for st in setups])
    b.close()
    for got, ref in zip(outs[0], plain):
        assert np.abs(got - ref).max() / np.abs(ref).max() <= 1e-5
    for a, c in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, c)
    _say(f"tuned batch kept the {'persistent' if form else 'graph'} form")
    given = _planes_case(**_persistent_cases()[6])
    ref = _plain(given)
    b = api.Batch([(given["dec"].ctx, given["obs"], given["est"], given["run"])], tune=True)
    assert b.info()["persistent"] and b.form_times() == (0.0, 0.0)
    _reset(given)
    b.launch()
    b.wait()
    np.testing.assert_array_equal(given["est"].cpu().numpy(), ref)
    b.close()
    for st in setups + [given]:
        st["dec"].close()
