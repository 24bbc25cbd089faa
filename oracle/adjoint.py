"""FP64 reverse sweep (adjoint) of the unrolled multi-view RL iterations.

TEST INFRASTRUCTURE ONLY (same rules as ``oracle.mvrl``).

The forward map is the update of Supplementary Note 1 with the back-projector
of Supplementary Note 2 §1, with view weights tempering each correction:

    b_v = ψ ⊛ P_v,  r_v = φ_v / b_v (1 where b_v ≤ ε),  q_v = r_v ⊛ X_v,
    c_v = w_v q_v + (1 − w_v),  ψ' = ψ · Π_v c_v            (simultaneous)
    ψ ← ψ · c_v(ψ)  for v = 0 … V−1                          (sequential)

Given ∂L/∂ψ^T this module returns ∂L/∂P_v, ∂L/∂X_v (K×K taps), ∂L/∂w_v and
∂L/∂ψ^0 by running the chain rule backwards through every step, recomputing the
intermediates of iteration t from the stored ψ^t (per-iteration checkpoints).
A weight w_v may be a per-pixel array (the per-pixel, per-view weights of the
memory table in Supplementary Note 2, read as the same tempering pixel by
pixel); its gradient is then the per-pixel array ∂L/∂w_v(pixel) = Σ_t c̄_v·(q_v − 1)
instead of that array's sum.

With the EM-normalised back-projection (``normalize``: q_v / s_v where
s_v = 1 ⊛ X_v > ε, see ``mvrl.view_factor``) the chain rule also runs through
s_v: q̄ = q̄'/s_v and s̄_v = −q̄'·q'/s_v where s_v > ε, and since s_v is the
convolution of a plane of ones with X_v, ∂L/∂X_v gains the tap gradient of s̄_v
against that plane.

Tap derivatives follow from differentiating the convolution sum
(a ⊛ k)[z][x] = Σ k[j][i] ã[z+Rz−j][x+Rx−i]:  ∂/∂k[j][i] = ã[z+Rz−j][x+Rx−i],
so ∂L/∂k[j][i] = Σ_{z,x} ḡ[z][x] ã[z+Rz−j][x+Rx−i] for the upstream gradient ḡ.
The adjoint of a ⊛ k in a is ḡ ⊛ flip(k) (both boundaries).
"""
from __future__ import annotations

import numpy as np

from .mvrl import EPS, PERIODIC, SEQUENTIAL, SIMULTANEOUS, ZERO, _extend, conv2d, flip, ratio, sensitivity


def tap_gradient(gbar, a, kshape, boundary=ZERO) -> np.ndarray:
    """∂L/∂k for y = a ⊛ k given ḡ = ∂L/∂y, summed over all planes (leading axes)."""
    kz, kx = kshape
    rz, rx = (kz - 1) // 2, (kx - 1) // 2
    nz, nx = a.shape[-2], a.shape[-1]
    ext = _extend(np.asarray(a, dtype=np.float64), rz, rx, boundary)
    out = np.zeros((kz, kx))
    for j in range(kz):
        for i in range(kx):
            out[j, i] = np.sum(gbar * ext[..., 2 * rz - j: 2 * rz - j + nz, 2 * rx - i: 2 * rx - i + nx])
    return out


def _factors(psi, phis, psfs, backs, ws, boundary, method="direct", normalize=False):
    """b, mask, r, q, c, s of every view from the same ψ (q normalised by the
    sensitivity s where s > ε when ``normalize``; s None otherwise)."""
    out = []
    for phi, p, x, w in zip(phis, psfs, backs, ws):
        b = conv2d(psi, p, boundary, method)
        m = b > EPS
        r = ratio(phi, b)
        q = conv2d(r, x, boundary, method)
        sens = None
        if normalize:
            sens = sensitivity(psi.shape[-2:], x, boundary, method)
            q = np.where(sens > EPS, q / np.where(sens > EPS, sens, 1.0), q)
        c = w * q + (1.0 - w)
        out.append((b, m, r, q, c, sens))
    return out


def _view_adjoint(cbar, psi, phi_parts, p, x, w, boundary, gp, gx, method="direct"):
    """Back-propagate c̄ of one view into ψ̄ (returned) and the tap/weight gradients."""
    b, m, r, q, _, sens = phi_parts
    # ∂c/∂w = q − 1, pixel by pixel; a scalar weight collects the sum
    gw = cbar * (q - 1.0) if np.ndim(w) else float(np.sum(cbar * (q - 1.0)))
    qbar = w * cbar
    if sens is not None:
        # q = q_raw / s where s > ε: q̄_raw = q̄ / s, s̄ = −q̄ · q / s; s = 1 ⊛ X
        ok = sens > EPS
        safe = np.where(ok, sens, 1.0)
        sbar = np.where(ok, -qbar * q / safe, 0.0)
        qbar = np.where(ok, qbar / safe, qbar)
        gx += tap_gradient(sbar, np.ones_like(psi), x.shape, boundary)
    rbar = conv2d(qbar, flip(x), boundary, method)
    gx += tap_gradient(qbar, r, x.shape, boundary)
    safe = np.where(m, b, 1.0)
    bbar = np.where(m, -rbar * r / safe, 0.0)
    psibar = conv2d(bbar, flip(p), boundary, method)
    gp += tap_gradient(bbar, psi, p.shape, boundary)
    return psibar, gw


def forward_history(phis, psfs, backs, weights, iters, update=SIMULTANEOUS, boundary=ZERO, psi0=None,
                    method="direct", normalize=False):
    """[ψ^0, …, ψ^T] with ψ^0 the mean of the observations unless given."""
    from .mvrl import init_estimate, rl_iteration

    psi = init_estimate(phis) if psi0 is None else np.asarray(psi0, dtype=np.float64)
    hist = [psi]
    for _ in range(iters):
        psi = rl_iteration(psi, phis, psfs, backs, weights, update, boundary, method, normalize)
        hist.append(psi)
    return hist


def adjoint(phis, psfs, backs, weights, iters, grad_out, update=SIMULTANEOUS, boundary=ZERO,
            psi0=None, history=None, method="direct", normalize=False):
    """Reverse sweep.  Returns dict(grad_psf=[V×K×K], grad_back=[V×K×K],
    grad_weights=[V], grad_psi0=array).  With a per-pixel weight array among
    the weights, grad_weights is a list whose entry v is a float for a scalar
    w_v and an array of w_v's shape for an array w_v."""
    nv = len(phis)
    ps = [np.asarray(p, dtype=np.float64) for p in psfs]
    xs = [np.asarray(x, dtype=np.float64) for x in backs]
    ws = [1.0] * nv if weights is None else [np.asarray(w, dtype=np.float64) if np.ndim(w) else float(w)
                                             for w in weights]
    per_pixel = any(np.ndim(w) for w in ws)
    hist = history if history is not None else forward_history(phis, ps, xs, ws, iters, update, boundary, psi0,
                                                               method, normalize)
    gp = [np.zeros_like(p) for p in ps]
    gx = [np.zeros_like(x) for x in xs]
    gw = [0.0] * nv
    gbar = np.asarray(grad_out, dtype=np.float64).copy()
    for t in range(iters - 1, -1, -1):
        psi = hist[t]
        if update == SIMULTANEOUS:
            parts = _factors(psi, phis, ps, xs, ws, boundary, method, normalize)
            cs = [pt[4] for pt in parts]
            prod = np.ones_like(psi)
            for c in cs:
                prod = prod * c
            new = gbar * prod
            for v in range(nv):
                others = np.ones_like(psi)
                for u in range(nv):
                    if u != v:
                        others = others * cs[u]
                cbar = gbar * psi * others
                pb, g = _view_adjoint(cbar, psi, parts[v], ps[v], xs[v], ws[v], boundary, gp[v], gx[v], method)
                new = new + pb
                gw[v] += g
            gbar = new
        elif update == SEQUENTIAL:
            sub = [psi]
            parts = []
            for v in range(nv):
                pt = _factors(sub[-1], [phis[v]], [ps[v]], [xs[v]], [ws[v]], boundary, method, normalize)[0]
                parts.append(pt)
                sub.append(sub[-1] * pt[4])
            for v in range(nv - 1, -1, -1):
                cur = sub[v]
                cbar = gbar * cur
                pb, g = _view_adjoint(cbar, cur, parts[v], ps[v], xs[v], ws[v], boundary, gp[v], gx[v], method)
                gbar = gbar * parts[v][4] + pb
                gw[v] += g
        else:
            raise ValueError(update)
    return dict(grad_psf=gp, grad_back=gx, grad_weights=list(gw) if per_pixel else np.array(gw), grad_psi0=gbar)


# ---------------------------------------------------------------------------
# Gaussian PSF parametrisation and the chain to (σx, σz)
# ---------------------------------------------------------------------------
def gaussian_taps(k, sigma_x, sigma_z):
    """Normalised point-sampled Gaussian (rows Z, columns X) and its derivatives
    with respect to σx and σz (normalisation included)."""
    d = np.arange(k, dtype=np.float64) - (k - 1) / 2.0
    gx = np.exp(-d * d / (2 * sigma_x ** 2))
    gz = np.exp(-d * d / (2 * sigma_z ** 2))
    dgx = gx * d * d / sigma_x ** 3
    dgz = gz * d * d / sigma_z ** 3
    sx, sz = gx.sum(), gz.sum()
    nx, nz = gx / sx, gz / sz
    dnx = dgx / sx - gx * dgx.sum() / sx ** 2
    dnz = dgz / sz - gz * dgz.sum() / sz ** 2
    return np.outer(nz, nx), np.outer(nz, dnx), np.outer(dnz, nx)


def mse_loss_and_grad(psi, truth):
    n = psi.size
    d = psi - truth
    return float(np.sum(d * d) / n), 2.0 * d / n


def sigma_gradients(phis, sigmas, weights, iters, truth, k, update=SIMULTANEOUS, boundary=ZERO):
    """Loss MSE(ψ^T, truth) with P_v = Gaussian(σ_v), X_v = P_v^*; returns
    (loss, dL/dσ [V×2 as (σx, σz)], dL/dw [V])."""
    taps = [gaussian_taps(k, sx, sz) for sx, sz in sigmas]
    ps = [t[0] for t in taps]
    xs = [flip(p) for p in ps]
    hist = forward_history(phis, ps, xs, weights, iters, update, boundary)
    loss, g = mse_loss_and_grad(hist[-1], truth)
    res = adjoint(phis, ps, xs, weights, iters, g, update, boundary, history=hist)
    gs = np.zeros((len(sigmas), 2))
    for v, (p, dpx, dpz) in enumerate(taps):
        total = res["grad_psf"][v] + flip(res["grad_back"][v])   # X_v = flip(P_v)
        gs[v, 0] = np.sum(total * dpx)
        gs[v, 1] = np.sum(total * dpz)
    return loss, gs, res["grad_weights"]


def sigma_loss(phis, sigmas, weights, iters, truth, k, update=SIMULTANEOUS, boundary=ZERO):
    ps = [gaussian_taps(k, sx, sz)[0] for sx, sz in sigmas]
    xs = [flip(p) for p in ps]
    psi = forward_history(phis, ps, xs, weights, iters, update, boundary)[-1]
    return mse_loss_and_grad(psi, truth)[0]
