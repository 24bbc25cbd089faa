"""Pins of the oracle's reverse sweep: central finite differences in FP64,
PyTorch CPU float64 autograd through an independent restatement of the forward
map (torch's own convolution), and exact zeros where a view's weight is 0.
Per-pixel weight arrays are pinned the same ways, and a constant array must
give, summed, the scalar weight's gradient; so is the EM-normalised
back-projection (whose sensitivity 1 ⊛ X_v depends on the back-projector's
taps)."""
import numpy as np
import pytest

import oracle
from oracle import adjoint as A
from synthetic import random_psf


def _problem(seed, shape=(2, 10, 9), kshapes=((5, 3), (3, 5)), weights=(0.8, 0.6)):
    rng = np.random.default_rng(seed)
    phis = [rng.uniform(20.0, 120.0, shape) for _ in kshapes]
    psfs = [random_psf(rng, kz, kx) for kz, kx in kshapes]
    backs = [random_psf(rng, kz, kx) for kz, kx in kshapes]
    gout = rng.standard_normal(shape)
    return phis, psfs, backs, list(weights), gout


def _loss(phis, psfs, backs, ws, T, gout, update, boundary, normalize=False):
    psi = A.forward_history(phis, psfs, backs, ws, T, update, boundary, normalize=normalize)[-1]
    return float(np.sum(gout * psi))


@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_adjoint_matches_central_differences(update, boundary):
    phis, psfs, backs, ws, gout = _problem(1)
    T = 3
    res = A.adjoint(phis, psfs, backs, ws, T, gout, update, boundary)
    rng = np.random.default_rng(2)
    h = 1e-6
    for v in range(2):
        for which, taps, grad in (("psf", psfs, res["grad_psf"]), ("back", backs, res["grad_back"])):
            for _ in range(4):
                j = rng.integers(taps[v].shape[0])
                i = rng.integers(taps[v].shape[1])
                plus = [t.copy() for t in taps]
                minus = [t.copy() for t in taps]
                plus[v][j, i] += h
                minus[v][j, i] -= h
                if which == "psf":
                    lp = _loss(phis, plus, backs, ws, T, gout, update, boundary)
                    lm = _loss(phis, minus, backs, ws, T, gout, update, boundary)
                else:
                    lp = _loss(phis, psfs, plus, ws, T, gout, update, boundary)
                    lm = _loss(phis, psfs, minus, ws, T, gout, update, boundary)
                fd = (lp - lm) / (2 * h)
                scale = max(1.0, np.abs(grad[v]).max())
                assert abs(fd - grad[v][j, i]) <= 1e-6 * scale, (which, v, j, i, fd, grad[v][j, i])
        wp = list(ws); wm = list(ws)
        wp[v] += h
        wm[v] -= h
        fd = (_loss(phis, psfs, backs, wp, T, gout, update, boundary)
              - _loss(phis, psfs, backs, wm, T, gout, update, boundary)) / (2 * h)
        assert abs(fd - res["grad_weights"][v]) <= 1e-6 * max(1.0, abs(fd))


def _torch_forward(torch, phis, psfs, backs, ws, T, update, boundary, normalize=False, psi0=None):
    """The forward map restated with torch.nn.functional.conv2d (a correlation:
    convolving with k is correlating with flip(k)); ``normalize`` divides each
    back-projection by 1 ⊛ X_v where that exceeds ε."""
    F = torch.nn.functional

    def conv(a, k):
        kz, kx = k.shape
        rz, rx = (kz - 1) // 2, (kx - 1) // 2
        x = a.unsqueeze(1)
        if boundary == "zero":
            x = F.pad(x, (rx, rx, rz, rz))
        else:
            x = F.pad(x, (rx, rx, rz, rz), mode="circular")
        return F.conv2d(x, torch.flip(k, (0, 1)).reshape(1, 1, kz, kx)).squeeze(1)

    def back(r, x):
        q = conv(r, x)
        if normalize:
            sens = conv(torch.ones_like(r), x)
            ok = sens > oracle.EPS
            q = torch.where(ok, q / torch.where(ok, sens, torch.ones_like(sens)), q)
        return q

    psi = sum(phis) / len(phis) if psi0 is None else psi0
    for _ in range(T):
        if update == "simultaneous":
            prod = torch.ones_like(psi)
            for phi, p, x, w in zip(phis, psfs, backs, ws):
                b = conv(psi, p)
                r = torch.where(b > oracle.EPS, phi / torch.where(b > oracle.EPS, b, torch.ones_like(b)),
                                torch.ones_like(b))
                prod = prod * (w * back(r, x) + (1 - w))
            psi = psi * prod
        else:
            for phi, p, x, w in zip(phis, psfs, backs, ws):
                b = conv(psi, p)
                r = torch.where(b > oracle.EPS, phi / torch.where(b > oracle.EPS, b, torch.ones_like(b)),
                                torch.ones_like(b))
                psi = psi * (w * back(r, x) + (1 - w))
    return psi


@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_adjoint_matches_torch_autograd(update, boundary):
    torch = pytest.importorskip("torch")
    phis, psfs, backs, ws, gout = _problem(3, shape=(2, 8, 11), kshapes=((3, 5), (5, 3), (3, 3)),
                                           weights=(1.0, 0.7, 0.5))
    T = 2
    res = A.adjoint(phis, psfs, backs, ws, T, gout, update, boundary)
    tphis = [torch.tensor(p, dtype=torch.float64) for p in phis]
    tp = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in psfs]
    tx = [torch.tensor(x, dtype=torch.float64, requires_grad=True) for x in backs]
    tw = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in ws]
    psi = _torch_forward(torch, tphis, tp, tx, tw, T, update, boundary)
    (psi * torch.tensor(gout)).sum().backward()
    for v in range(3):
        np.testing.assert_allclose(res["grad_psf"][v], tp[v].grad.numpy(), rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(res["grad_back"][v], tx[v].grad.numpy(), rtol=1e-10, atol=1e-12)
        assert abs(res["grad_weights"][v] - tw[v].grad.item()) <= 1e-10 * max(1.0, abs(tw[v].grad.item()))


def test_zero_weight_gives_zero_tap_gradients():
    phis, psfs, backs, ws, gout = _problem(4, weights=(0.0, 0.9))
    for update in ("simultaneous", "sequential"):
        res = A.adjoint(phis, psfs, backs, ws, 3, gout, update)
        assert np.all(res["grad_psf"][0] == 0.0) and np.all(res["grad_back"][0] == 0.0)
        assert np.any(res["grad_psf"][1] != 0.0)


def test_sigma_gradients_match_central_differences():
    """MSE to a truth through Gaussian PSFs: σ and weight gradients vs FP64
    central differences with h = 1e-4."""
    rng = np.random.default_rng(5)
    shape = (2, 20, 18)
    truth = 100.0 + 600.0 * (rng.random(shape) > 0.95)
    k = 11
    data_sig = [(1.5, 3.0), (3.0, 1.5)]
    phis = [oracle.conv2d(truth, A.gaussian_taps(k, *s)[0]) + rng.uniform(0, 2, shape) for s in data_sig]
    sig = [(1.7, 3.3), (3.2, 1.6)]
    ws = [0.9, 0.8]
    loss, gs, gw = A.sigma_gradients(phis, sig, ws, 3, truth, k)
    h = 1e-4
    for v in range(2):
        for a in range(2):
            sp = [list(s) for s in sig]
            sm = [list(s) for s in sig]
            sp[v][a] += h
            sm[v][a] -= h
            fd = (A.sigma_loss(phis, sp, ws, 3, truth, k) - A.sigma_loss(phis, sm, ws, 3, truth, k)) / (2 * h)
            assert abs(fd - gs[v, a]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gs).max()), (v, a, fd, gs[v, a])
        wp = list(ws); wm = list(ws)
        wp[v] += h
        wm[v] -= h
        fd = (A.sigma_loss(phis, sig, wp, 3, truth, k) - A.sigma_loss(phis, sig, wm, 3, truth, k)) / (2 * h)
        assert abs(fd - gw[v]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gw).max())


def test_gaussian_derivative_taps_match_differences():
    k, sx, sz = 9, 1.6, 2.7
    p, dpx, dpz = A.gaussian_taps(k, sx, sz)
    h = 1e-6
    np.testing.assert_allclose(dpx, (A.gaussian_taps(k, sx + h, sz)[0] - A.gaussian_taps(k, sx - h, sz)[0]) / (2 * h),
                               atol=1e-9)
    np.testing.assert_allclose(dpz, (A.gaussian_taps(k, sx, sz + h)[0] - A.gaussian_taps(k, sx, sz - h)[0]) / (2 * h),
                               atol=1e-9)
    from synthetic import gaussian_psf
    np.testing.assert_allclose(p, gaussian_psf(k, sx, sz), rtol=1e-14)


def _pixel_weights(seed, shape, nv):
    rng = np.random.default_rng(seed)
    return [rng.uniform(0.3, 1.0, shape) for _ in range(nv)]


@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_pixel_weight_gradients_match_central_differences(update, boundary):
    phis, psfs, backs, _, gout = _problem(5)
    ws = _pixel_weights(6, gout.shape, 2)
    T = 3
    res = A.adjoint(phis, psfs, backs, ws, T, gout, update, boundary)
    assert isinstance(res["grad_weights"], list) and res["grad_weights"][0].shape == gout.shape
    rng = np.random.default_rng(7)
    h = 1e-6
    for v in range(2):
        scale = max(1.0, np.abs(res["grad_weights"][v]).max())
        for _ in range(5):
            idx = tuple(int(rng.integers(n)) for n in gout.shape)
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[v][idx] += h
            wm[v][idx] -= h
            fd = (_loss(phis, psfs, backs, wp, T, gout, update, boundary)
                  - _loss(phis, psfs, backs, wm, T, gout, update, boundary)) / (2 * h)
            assert abs(fd - res["grad_weights"][v][idx]) <= 1e-6 * scale, (v, idx, fd, res["grad_weights"][v][idx])
        # the taps' gradients under per-pixel weights
        j, i = 1, 2
        plus = [t.copy() for t in psfs]
        minus = [t.copy() for t in psfs]
        plus[v][j, i] += h
        minus[v][j, i] -= h
        fd = (_loss(phis, plus, backs, ws, T, gout, update, boundary)
              - _loss(phis, minus, backs, ws, T, gout, update, boundary)) / (2 * h)
        assert abs(fd - res["grad_psf"][v][j, i]) <= 1e-6 * max(1.0, np.abs(res["grad_psf"][v]).max())


@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
def test_pixel_weight_gradients_match_torch_autograd(update):
    torch = pytest.importorskip("torch")
    phis, psfs, backs, _, gout = _problem(8, shape=(2, 8, 11), kshapes=((3, 5), (5, 3), (3, 3)))
    ws = _pixel_weights(9, gout.shape, 3)
    ws[1] = 0.7                       # scalar and per-pixel weights mixed
    T = 2
    res = A.adjoint(phis, psfs, backs, ws, T, gout, update, "zero")
    tphis = [torch.tensor(p, dtype=torch.float64) for p in phis]
    tp = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in psfs]
    tx = [torch.tensor(x, dtype=torch.float64, requires_grad=True) for x in backs]
    tw = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in ws]
    psi = _torch_forward(torch, tphis, tp, tx, tw, T, update, "zero")
    (psi * torch.tensor(gout)).sum().backward()
    for v in range(3):
        np.testing.assert_allclose(res["grad_psf"][v], tp[v].grad.numpy(), rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(res["grad_back"][v], tx[v].grad.numpy(), rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(res["grad_weights"][v], tw[v].grad.numpy(), rtol=1e-10, atol=1e-12)
    assert np.ndim(res["grad_weights"][1]) == 0


def test_constant_pixel_weights_sum_to_the_scalar_gradient():
    phis, psfs, backs, _, gout = _problem(10)
    for update in ("simultaneous", "sequential"):
        scal = A.adjoint(phis, psfs, backs, [0.8, 0.6], 3, gout, update)
        arr = A.adjoint(phis, psfs, backs, [np.full(gout.shape, 0.8), np.full(gout.shape, 0.6)], 3, gout, update)
        for v in range(2):
            assert abs(arr["grad_weights"][v].sum() - scal["grad_weights"][v]) <= 1e-9 * max(
                1.0, abs(scal["grad_weights"][v]))
            np.testing.assert_allclose(arr["grad_psf"][v], scal["grad_psf"][v], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(arr["grad_psi0"], scal["grad_psi0"], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_normalised_adjoint_matches_central_differences(update, boundary):
    """EM-normalised back-projection: every gradient against FP64 central
    differences, the back-projector's taps included (they enter through the
    sensitivity 1 ⊛ X_v as well as through the back-projection)."""
    phis, psfs, backs, ws, gout = _problem(11)
    T = 3
    res = A.adjoint(phis, psfs, backs, ws, T, gout, update, boundary, normalize=True)
    rng = np.random.default_rng(12)
    h = 1e-6
    for v in range(2):
        for which, taps, grad in (("psf", psfs, res["grad_psf"]), ("back", backs, res["grad_back"])):
            scale = max(1.0, np.abs(grad[v]).max())
            for _ in range(4):
                j = int(rng.integers(taps[v].shape[0]))
                i = int(rng.integers(taps[v].shape[1]))
                plus = [t.copy() for t in taps]
                minus = [t.copy() for t in taps]
                plus[v][j, i] += h
                minus[v][j, i] -= h
                if which == "psf":
                    lp = _loss(phis, plus, backs, ws, T, gout, update, boundary, True)
                    lm = _loss(phis, minus, backs, ws, T, gout, update, boundary, True)
                else:
                    lp = _loss(phis, psfs, plus, ws, T, gout, update, boundary, True)
                    lm = _loss(phis, psfs, minus, ws, T, gout, update, boundary, True)
                fd = (lp - lm) / (2 * h)
                assert abs(fd - grad[v][j, i]) <= 1e-6 * scale, (which, v, j, i, fd, grad[v][j, i])
        wp = list(ws)
        wm = list(ws)
        wp[v] += h
        wm[v] -= h
        fd = (_loss(phis, psfs, backs, wp, T, gout, update, boundary, True)
              - _loss(phis, psfs, backs, wm, T, gout, update, boundary, True)) / (2 * h)
        assert abs(fd - res["grad_weights"][v]) <= 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_normalised_adjoint_matches_torch_autograd(update, boundary):
    torch = pytest.importorskip("torch")
    phis, psfs, backs, ws, gout = _problem(13, shape=(2, 8, 11), kshapes=((3, 5), (5, 3), (3, 3)),
                                           weights=(1.0, 0.7, 0.5))
    T = 2
    res = A.adjoint(phis, psfs, backs, ws, T, gout, update, boundary, normalize=True)
    tphis = [torch.tensor(p, dtype=torch.float64) for p in phis]
    tp = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in psfs]
    tx = [torch.tensor(x, dtype=torch.float64, requires_grad=True) for x in backs]
    tw = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in ws]
    t0 = (sum(tphis) / len(tphis)).detach().requires_grad_(True)
    psi = _torch_forward(torch, tphis, tp, tx, tw, T, update, boundary, normalize=True, psi0=t0)
    (psi * torch.tensor(gout)).sum().backward()
    for v in range(3):
        np.testing.assert_allclose(res["grad_psf"][v], tp[v].grad.numpy(), rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(res["grad_back"][v], tx[v].grad.numpy(), rtol=1e-10, atol=1e-12)
        assert abs(res["grad_weights"][v] - tw[v].grad.item()) <= 1e-10 * max(1.0, abs(tw[v].grad.item()))
    np.testing.assert_allclose(res["grad_psi0"], t0.grad.numpy(), rtol=1e-10, atol=1e-12)
