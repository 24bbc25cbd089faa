"""Differentiable plane-wise MV-RL: ψ^T as a function of per-view Gaussian PSF
widths (σx, σz) or of the PSF taps themselves (measured PSFs of any rank),
the view weights and, optionally, per-pixel weight planes, behind
``torch.autograd.Function``.

Forward: the HIP library runs the unrolled RL iterations and stores ψ^t of
every iteration (checkpoints).  Backward: the library's reverse sweep
(``mvd_backward_grads``) returns ∂L/∂P_v and ∂L/∂X_v on the K×K taps, ∂L/∂w_v
and ∂L/∂ω_v of the weight planes; with X_v = P_v^* the tap gradient of P_v is
∂L/∂P_v + flip(∂L/∂X_v), chained to (σx, σz) by torch through the small
Gaussian builder (K×K values, float64).  The EM-normalised back-projection
(``normalize=True``) is differentiated too.
"""
from __future__ import annotations

import numpy as np

from . import api


def _torch():
    import torch
    return torch


def gaussian_taps(k: int, sigma_x, sigma_z):
    """Normalised point-sampled Gaussian [K][K] (rows Z, columns X), float64, differentiable."""
    torch = _torch()
    d = torch.arange(k, dtype=torch.float64, device=sigma_x.device) - (k - 1) / 2.0
    gx = torch.exp(-d * d / (2 * sigma_x * sigma_x))
    gz = torch.exp(-d * d / (2 * sigma_z * sigma_z))
    p = gz[:, None] * gx[None, :]
    return p / p.sum()


class PlanewiseRL:
    """Observations and run settings of one differentiable deconvolution."""

    def __init__(self, obs, k: int, iters: int, *, update="simultaneous", boundary="zero",
                 layout="stack_zyx", device: int = 0, normalize: bool = False):
        torch = _torch()
        self.obs = list(obs)
        self.k, self.iters, self.update, self.boundary, self.layout = k, iters, update, boundary, layout
        self.normalize = normalize
        o0 = self.obs[0]
        if layout == "stack_zyx":
            self.nz, self.ny, self.nx = o0.shape[0], o0.shape[1], o0.shape[2]
        else:
            self.ny, self.nz, self.nx = o0.shape
        self.obs_dtype = "u16" if o0.dtype == torch.uint16 else "f32"
        self.dec = api.Deconvolver(len(self.obs), self.nz, self.nx, device)
        self.dev = o0.device
        self.timing = False   # record per-launch HIP events (read with api.mvd_get_timing)
        self._sigma_set = None   # the (σx, σz) values whose taps the context holds

    def _run(self, weights, checkpoints=None, ws_bytes=0, tune=False, planes=None):
        return api.make_run(self.ny, self.iters, update=self.update, boundary=self.boundary,
                            obs_dtype=self.obs_dtype, layout=self.layout, weights=weights,
                            checkpoints=checkpoints, timing=self.timing, tune=tune, normalize=self.normalize,
                            weight_planes=[planes[v] for v in range(planes.shape[0])] if planes is not None
                            else None)

    def set_sigmas(self, sigma):
        """Give the context the taps of these widths (no-op if it holds them already)."""
        s = sigma.detach().to("cpu", dtype=_torch().float64)
        key = ("sigma",) + tuple(s.flatten().tolist())
        if key == self._sigma_set:
            return
        self._sigma_set = None
        for v in range(len(self.obs)):
            taps = gaussian_taps(self.k, s[v, 0], s[v, 1]).numpy().astype(np.float32)
            self.dec.set_psf(v, taps, "flipped")
        self._sigma_set = key

    def set_taps(self, taps):
        """Give the context these PSF taps, [V][K][K] (no-op if it holds them already)."""
        t = taps.detach().to("cpu", dtype=_torch().float64)
        key = ("taps",) + tuple(t.flatten().tolist())
        if key == self._sigma_set:
            return
        self._sigma_set = None
        for v in range(len(self.obs)):
            self.dec.set_psf(v, t[v].numpy().astype(np.float32), "flipped")
        self._sigma_set = key

    def __call__(self, sigma, weights, weight_planes=None):
        return mv_deconvolve(sigma, weights, self, weight_planes)


def _make_function():
    torch = _torch()

    def set_psfs(prob, params, taps_mode):
        if taps_mode:
            prob.set_taps(params)
        else:
            prob.set_sigmas(params)

    class MVDeconvFunction(torch.autograd.Function):
        """ψ^T(σ or taps, w, ω): forward and reverse sweep in the HIP library."""

        @staticmethod
        def forward(ctx, params, weights, planes, prob: PlanewiseRL, taps_mode: bool):
            set_psfs(prob, params, taps_mode)
            w = [float(x) for x in weights.detach().cpu().tolist()]
            T = prob.iters
            pl = planes.detach().float().contiguous() if planes is not None else None
            ck = torch.empty((T, prob.ny, prob.nz, prob.nx), dtype=torch.float32, device=prob.dev)
            est = torch.empty((prob.ny, prob.nz, prob.nx), dtype=torch.float32, device=prob.dev)
            # launch shapes timed on the first call for this workload (cached by the
            # library, which reuses them for the reverse sweep)
            run = prob._run(w, checkpoints=ck.data_ptr(), tune=not prob.timing, planes=pl)
            nbytes = api.mvd_workspace_bytes(prob.dec.ctx, run)
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=prob.dev)
            run.workspace = (ws.data_ptr() + 255) // 256 * 256
            run.workspace_bytes = nbytes
            api.mvd_deconvolve_planes(prob.dec.ctx, prob.obs, est, run)
            ctx.prob = prob
            ctx.w = w
            ctx.taps_mode = taps_mode
            ctx.has_planes = pl is not None
            ctx.save_for_backward(params, weights, ck, *((pl,) if pl is not None else ()))
            return est

        @staticmethod
        def backward(ctx, grad_out):
            params, weights, ck = ctx.saved_tensors[:3]
            pl = ctx.saved_tensors[3] if ctx.has_planes else None
            prob = ctx.prob
            # the reverse sweep recomputes every iteration with the context's taps: give it
            # this forward's (another forward may have run in between, as gradcheck does)
            set_psfs(prob, params, ctx.taps_mode)
            V, K = len(prob.obs), prob.k
            run = prob._run(ctx.w, checkpoints=ck.data_ptr(), planes=pl)
            nbytes = api.mvd_backward_workspace_bytes(prob.dec.ctx, run)
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=prob.dev)
            run.workspace = (ws.data_ptr() + 255) // 256 * 256
            run.workspace_bytes = nbytes
            gp = [torch.empty((K, K), dtype=torch.float32, device=prob.dev) for _ in range(V)]
            gb = [torch.empty((K, K), dtype=torch.float32, device=prob.dev) for _ in range(V)]
            gw = torch.empty(V, dtype=torch.float32, device=prob.dev)
            gwp = None
            if pl is not None and ctx.needs_input_grad[2]:
                gwp = torch.empty_like(pl)
            api.mvd_backward_grads(prob.dec.ctx, prob.obs, grad_out.contiguous().float(), run, gp, gb, gw,
                                   None, [gwp[v] for v in range(V)] if gwp is not None else None)
            torch.cuda.current_stream().synchronize()
            grad_params = None
            if ctx.needs_input_grad[0]:
                tap_grads = [gp[v].double().cpu() + torch.flip(gb[v].double().cpu(), (0, 1)) for v in range(V)]
                if ctx.taps_mode:
                    grad_params = torch.stack(tap_grads).to(device=params.device, dtype=params.dtype)
                else:
                    with torch.enable_grad():
                        s = params.detach().to("cpu", dtype=torch.float64).requires_grad_(True)
                        total = 0.0
                        for v in range(V):
                            total = total + (gaussian_taps(K, s[v, 0], s[v, 1]) * tap_grads[v]).sum()
                        (g,) = torch.autograd.grad(total, s)
                    grad_params = g.to(device=params.device, dtype=params.dtype)
            grad_w = gw.to(device=weights.device, dtype=weights.dtype) if ctx.needs_input_grad[1] else None
            return grad_params, grad_w, gwp, None, None

    return MVDeconvFunction


_FUNCTION = None


def function_class():
    """The ``torch.autograd.Function`` subclass (created on first use)."""
    global _FUNCTION
    if _FUNCTION is None:
        _FUNCTION = _make_function()
    return _FUNCTION


def mv_deconvolve(sigma, weights, prob: PlanewiseRL, weight_planes=None):
    """ψ^T(σ, w[, ω]) with autograd support (σ: [V][2] as (σx, σz); w: [V];
    ω: per-pixel weight planes [V][Y][Z][X] on the device, or None)."""
    return function_class().apply(sigma, weights, weight_planes, prob, False)


def mv_deconvolve_taps(taps, weights, prob: PlanewiseRL, weight_planes=None):
    """ψ^T(P, w[, ω]) with autograd support for PSF taps given directly
    (taps: [V][K][K] with K = prob.k, any rank: rank-one, low-rank or K×K passes
    as the library finds; X_v = P_v^*)."""
    return function_class().apply(taps, weights, weight_planes, prob, True)
