"""Plain FP64 CPU oracle of plane-wise multi-view Richardson-Lucy deconvolution.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this module.  The GPU
library never calls it and shares no code with it.

Everything is float64 numpy, written in the paper's order and notation:

* the multi-view RL update ψ^{t+1} = ψ^t · Π_v [(φ_v / (ψ^t ∗ P_v)) ∗ X_v]
  (Supplementary Note 1, the update equation; Supplementary Note 2 §1 for the
  general back-projector X);
* X_v = P_v^* (the point-reflected PSF, "Independent") or one of the compound
  kernels of Supplementary Note 2 §1 (Efficient Bayesian, Optimization I and II);
* the plane-wise approximation: every plane orthogonal to the rotation axis is
  processed on its own with a 2D PSF (Results, second paragraph; Fig. 1a);
* convolution boundary: zero-extended linear convolution, i.e. what a Fourier
  convolution padded to data + PSF size computes (Supplementary Table 1 caption),
  or periodic as a second mode.

Readings where the paper is silent (initial estimate, division guard, update
order, view weights, compound-kernel formulas) are the ones listed in the design
notes; each function states the one it uses.
"""
from __future__ import annotations

import numpy as np

EPS = 1e-6           # division guard: r = φ/b if b > EPS else 1

ZERO = "zero"
PERIODIC = "periodic"
SIMULTANEOUS = "simultaneous"
SEQUENTIAL = "sequential"
BACK_MODES = ("flipped", "efficient_bayes", "opt1", "opt2", "explicit")


# ---------------------------------------------------------------------------
# Reslice (Fig. 1a; Results: one plane per camera line)
# ---------------------------------------------------------------------------
def reslice(stack) -> np.ndarray:
    """Camera-ordered stack ``[Z][Y][X]`` → planes ``[Y][Z][X]`` in float64.

    Plane y is the Z×X image formed by camera row y of every slice z (planes
    orthogonal to the rotation axis Y, one per camera line).  uint16 converts
    exactly; float observations are clamped below at 0 (``fmax``, so NaN → 0).
    """
    a = np.asarray(stack)
    if a.ndim != 3:
        raise ValueError("stack must be [Z][Y][X]")
    if a.dtype == np.uint16:
        f = a.astype(np.float64)
    else:
        f = np.fmax(a.astype(np.float64), 0.0)
    nz, ny, nx = f.shape
    out = np.empty((ny, nz, nx), dtype=np.float64)
    for y in range(ny):
        out[y] = f[:, y, :]
    return out


def load_planes(obs) -> np.ndarray:
    """Observations already in plane order ``[Y][Z][X]`` → float64 (same conversion)."""
    a = np.asarray(obs)
    if a.dtype == np.uint16:
        return a.astype(np.float64)
    return np.fmax(a.astype(np.float64), 0.0)


# ---------------------------------------------------------------------------
# 2D convolution in the plane (Supplementary Note 1: ψ ∗ P_v and (·) ∗ X)
# ---------------------------------------------------------------------------
def flip(k) -> np.ndarray:
    """P^*: point reflection of a kernel in both axes, ``k[Kz-1-j][Kx-1-i]``."""
    k = np.asarray(k, dtype=np.float64)
    return k[::-1, ::-1].copy()


def _check_kernel(k):
    k = np.asarray(k, dtype=np.float64)
    if k.ndim != 2 or k.shape[0] % 2 == 0 or k.shape[1] % 2 == 0:
        raise ValueError("kernels must be 2D with odd sides")
    return k


def _extend(a, rz, rx, boundary):
    """ã: ``a`` extended by rz rows and rx columns each side (zeros or wrap-around)."""
    if boundary == ZERO:
        pad = [(0, 0)] * (a.ndim - 2) + [(rz, rz), (rx, rx)]
        return np.pad(a, pad, mode="constant")
    if boundary == PERIODIC:
        nz, nx = a.shape[-2], a.shape[-1]
        zi = (np.arange(-rz, nz + rz)) % nz
        xi = (np.arange(-rx, nx + rx)) % nx
        return a[..., zi, :][..., :, xi]
    raise ValueError(f"unknown boundary {boundary!r}")


def conv2d(a, k, boundary: str = ZERO, method: str = "direct") -> np.ndarray:
    """(a ⊛ k)[z][x] = Σ_j Σ_i k[j][i] · ã[z+Rz−j][x+Rx−i] over the last two axes.

    ã is ``a`` inside the plane and 0 outside (ZERO) or ``a`` at indices taken
    modulo the plane size (PERIODIC).  The kernel centre is tap (Rz, Rx) with
    R = (K−1)/2.  ``method="fft"`` computes the same sum through the convolution
    theorem (scipy.fft), used only to reach large planes in reasonable time.
    """
    a = np.asarray(a, dtype=np.float64)
    k = _check_kernel(k)
    kz, kx = k.shape
    rz, rx = (kz - 1) // 2, (kx - 1) // 2
    if method == "fft":
        return _conv2d_fft(a, k, boundary)
    if method != "direct":
        raise ValueError(method)
    nz, nx = a.shape[-2], a.shape[-1]
    ext = _extend(a, rz, rx, boundary)   # ext[p][q] = ã[p - rz][q - rx]
    out = np.zeros_like(a)
    for j in range(kz):
        for i in range(kx):
            w = k[j, i]
            if w == 0.0:
                continue
            # ã[z + rz - j] = ext[z + 2rz - j]
            out += w * ext[..., 2 * rz - j: 2 * rz - j + nz, 2 * rx - i: 2 * rx - i + nx]
    return out


def _conv2d_fft(a, k, boundary):
    import scipy.fft as sfft

    kz, kx = k.shape
    rz, rx = (kz - 1) // 2, (kx - 1) // 2
    nz, nx = a.shape[-2], a.shape[-1]
    if boundary == ZERO:
        fz, fx = nz + kz - 1, nx + kx - 1
        fa = sfft.rfft2(a, s=(fz, fx), axes=(-2, -1))
        fk = sfft.rfft2(k, s=(fz, fx))
        full = sfft.irfft2(fa * fk, s=(fz, fx), axes=(-2, -1))
        return np.ascontiguousarray(full[..., rz:rz + nz, rx:rx + nx])
    if boundary == PERIODIC:
        kw = np.zeros((nz, nx))
        for j in range(kz):
            for i in range(kx):
                kw[(j - rz) % nz, (i - rx) % nx] += k[j, i]
        fa = sfft.rfft2(a, axes=(-2, -1))
        fk = sfft.rfft2(kw)
        return sfft.irfft2(fa * fk, s=(nz, nx), axes=(-2, -1))
    raise ValueError(f"unknown boundary {boundary!r}")


def conv_full(a, b) -> np.ndarray:
    """Full linear convolution of two small kernels: size (Ka+Kb−1) per axis."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = np.zeros((a.shape[0] + b.shape[0] - 1, a.shape[1] + b.shape[1] - 1))
    for j in range(a.shape[0]):
        for i in range(a.shape[1]):
            out[j:j + b.shape[0], i:i + b.shape[1]] += a[j, i] * b
    return out


def crop_center(a, kz: int, kx: int) -> np.ndarray:
    """C_K: the centred kz×kx window of an odd-sided kernel (zero-extended if smaller)."""
    a = np.asarray(a, dtype=np.float64)
    out = np.zeros((kz, kx))
    cz, cx = (a.shape[0] - 1) // 2, (a.shape[1] - 1) // 2
    rz, rx = (kz - 1) // 2, (kx - 1) // 2
    for j in range(kz):
        sj = cz - rz + j
        if 0 <= sj < a.shape[0]:
            for i in range(kx):
                si = cx - rx + i
                if 0 <= si < a.shape[1]:
                    out[j, i] = a[sj, si]
    return out


# ---------------------------------------------------------------------------
# Back-projectors X (Supplementary Note 2 §1)
# ---------------------------------------------------------------------------
def back_projector(psfs, v: int, mode: str = "flipped", explicit=None) -> np.ndarray:
    """X for view ``v``.

    * flipped ("Independent"): X = P_v^*.
    * efficient_bayes: X = N( P_v^* ⊙ Π_{w≠v} C( P_v^* ⊛ P_w ⊛ P_w^* ) ).
    * opt1 ("Optimization I"): X = N( P_v^* ⊙ Π_{w≠v} C( P_v^* ⊛ P_w ) ).
    * opt2 ("Optimization II"): X = N( (P_v^*)^{⊙V} ).
    * explicit: the given kernel, as is.

    ⊙ and the power are pixel-wise, ⊛ is the full linear convolution, C crops
    the centred window of P_v's size and N divides by the sum.  W_v is every
    view except v.  The printed compound formulas are garbled; these are the
    readings of them.
    """
    pv = _check_kernel(psfs[v])
    kz, kx = pv.shape
    fv = flip(pv)
    if mode == "flipped":
        return fv
    if mode == "explicit":
        if explicit is None:
            raise ValueError("explicit back-projector needs its taps")
        return _check_kernel(explicit).copy()
    nv = len(psfs)
    if mode == "opt2":
        x = fv ** nv
    elif mode in ("efficient_bayes", "opt1"):
        x = fv.copy()
        for w in range(nv):
            if w == v:
                continue
            pw = _check_kernel(psfs[w])
            c = conv_full(fv, pw)
            if mode == "efficient_bayes":
                c = conv_full(c, flip(pw))
            x = x * crop_center(c, kz, kx)
    else:
        raise ValueError(f"unknown back-projector mode {mode!r}")
    s = x.sum()
    if not s > 0.0:
        raise ValueError("compound back-projector has zero sum")
    return x / s


# ---------------------------------------------------------------------------
# Initial estimate (paper silent; averaging fusion of Fig. 1f as ψ^0)
# ---------------------------------------------------------------------------
def init_estimate(phis, mode: str = "mean", const: float = 1.0, given=None) -> np.ndarray:
    """ψ^0 = (1/V) Σ_v φ_v ("mean"), a constant, or a given estimate."""
    if mode == "mean":
        acc = np.zeros_like(phis[0])
        for p in phis:
            acc = acc + p
        return acc / len(phis)
    if mode == "const":
        return np.full_like(phis[0], float(const))
    if mode == "given":
        return np.asarray(given, dtype=np.float64).copy()
    raise ValueError(mode)


# ---------------------------------------------------------------------------
# One RL iteration (Supplementary Note 1 / Note 2 §1 update)
# ---------------------------------------------------------------------------
def ratio(phi, b):
    """r = φ / b where b > EPS, else 1 (neutral): the division guard."""
    safe = np.where(b > EPS, b, 1.0)
    return np.where(b > EPS, phi / safe, 1.0)


def sensitivity(shape, x, boundary, method="direct"):
    """s = 1 ⊛ X: the back-projection of a plane of ones, i.e. Aᵀ1 when X = Aᵀ.
    Under the zero boundary it falls below the tap sum within R of the edges."""
    return conv2d(np.ones(shape), x, boundary, method)


def view_factor(psi, phi, p, x, w, boundary, method="direct", normalize=False):
    """c_v = w · [(φ_v / (ψ ⊛ P_v)) ⊛ X_v] + (1 − w) for one view.

    normalize: the back-projection is divided by s = 1 ⊛ X_v where s > EPS
    (the EM form ψ · Aᵀ(φ/Aψ) / Aᵀ1 of the update for a zero-extended
    convolution, whose columns do not all sum to one near the edges; the
    paper's update assumes they do, Supplementary Note 1).
    """
    b = conv2d(psi, p, boundary, method)
    r = ratio(phi, b)
    q = conv2d(r, x, boundary, method)
    if normalize:
        s = sensitivity(psi.shape[-2:], x, boundary, method)
        q = np.where(s > EPS, q / np.where(s > EPS, s, 1.0), q)
    return w * q + (1.0 - w)


def rl_iteration(psi, phis, psfs, backs, weights=None, update=SIMULTANEOUS,
                 boundary=ZERO, method="direct", normalize=False) -> np.ndarray:
    """ψ^{t+1} from ψ^t.

    simultaneous: every view's factor from the same ψ^t, then ψ^t · Π_v c_v
    (the printed update).  sequential: for v in order, ψ ← ψ · c_v(ψ), each
    view's correction multiplied into the estimate before the next view.
    Weights w_v (default 1) temper each factor as w·q + (1 − w); a weight may
    be a per-pixel array (the per-pixel, per-view weights of the memory table,
    whose formula the paper leaves open: read here as the same tempering
    pixel by pixel).  normalize: see view_factor.
    """
    nv = len(phis)
    # a weight is a scalar or, per pixel, an array of the planes' shape
    ws = [1.0] * nv if weights is None else [w if np.ndim(w) else float(w) for w in weights]
    if update == SIMULTANEOUS:
        prod = np.ones_like(psi)
        for v in range(nv):
            prod = prod * view_factor(psi, phis[v], psfs[v], backs[v], ws[v], boundary, method, normalize)
        return psi * prod
    if update == SEQUENTIAL:
        cur = psi
        for v in range(nv):
            cur = cur * view_factor(cur, phis[v], psfs[v], backs[v], ws[v], boundary, method, normalize)
        return cur
    raise ValueError(update)


def deconvolve(obs, psfs, iters: int, *, update=SIMULTANEOUS, boundary=ZERO,
               back="flipped", back_taps=None, weights=None, init="mean",
               init_const=1.0, init_given=None, layout="stack_zyx",
               method="direct", return_history=False, normalize=False):
    """Plane-wise MV-RL: reslice, ψ^0, then ``iters`` iterations; returns ψ^T ``[Y][Z][X]``.

    ``obs``: per-view stacks ``[Z][Y][X]`` (layout "stack_zyx") or planes
    ``[Y][Z][X]`` (layout "planes_yzx"), uint16 or float.  ``psfs``: per-view
    taps ``[Kz][Kx]`` used as given.  With ``return_history`` the list
    [ψ^0, …, ψ^T] is returned as well.
    """
    if layout == "stack_zyx":
        phis = [reslice(o) for o in obs]
    elif layout == "planes_yzx":
        phis = [load_planes(o) for o in obs]
    else:
        raise ValueError(layout)
    ps = [_check_kernel(p) for p in psfs]
    bt = back_taps if back_taps is not None else [None] * len(ps)
    backs = [back_projector(ps, v, back, bt[v]) for v in range(len(ps))]
    psi = init_estimate(phis, init, init_const, init_given)
    hist = [psi]
    for _ in range(int(iters)):
        psi = rl_iteration(psi, phis, ps, backs, weights, update, boundary, method, normalize)
        if return_history:
            hist.append(psi)
    if return_history:
        return psi, hist
    return psi


# ---------------------------------------------------------------------------
# Diagnostics
# ---------------------------------------------------------------------------
def i_divergence(psi, phis, psfs, boundary=ZERO, method="direct") -> float:
    """Σ_v Σ [φ ln(φ/b) − φ + b] with b = ψ ⊛ P_v and 0·ln 0 = 0 (Csiszár I-divergence)."""
    total = 0.0
    for phi, p in zip(phis, psfs):
        b = conv2d(psi, p, boundary, method)
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(phi > 0, phi * np.log(np.where(phi > 0, phi, 1.0) / b), 0.0)
        total += float(np.sum(t - phi + b))
    return total


def flux(psi) -> float:
    return float(np.sum(psi))
