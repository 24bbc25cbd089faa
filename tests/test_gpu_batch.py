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
