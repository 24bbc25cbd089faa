"""FP64 CPU reference of full 3D multi-view Richardson-Lucy (test infrastructure only).

Only the test suite may import this module.  It serves the validation of the
plane-wise approximation: the paper deconvolves every plane orthogonal to the
rotation axis on its own with a 2D PSF (Results, second paragraph; Fig. 1a)
and reports that this is indistinguishable from full 3D deconvolution while
the PSF's extent along the rotation axis stays small (Supplementary Figs. 2-4).
Here the same update equation (Supplementary Note 1) runs with 3D kernels over
the volume in plane order ``[Y][Z][X]``, zero-extended in all three axes.
"""
from __future__ import annotations

import numpy as np
import scipy.signal

from .mvrl import EPS, ratio


def conv3d(a, k) -> np.ndarray:
    """(a ⊛ k)[y][z][x] = Σ_{l,j,i} k[l][j][i] · ã[y+Ry−l][z+Rz−j][x+Rx−i], ã zero
    outside the volume; the 3D counterpart of the plane convolution."""
    a = np.asarray(a, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    ky, kz, kx = k.shape
    ry, rz, rx = (ky - 1) // 2, (kz - 1) // 2, (kx - 1) // 2
    ny, nz, nx = a.shape
    ext = np.zeros((ny + 2 * ry, nz + 2 * rz, nx + 2 * rx))
    ext[ry:ry + ny, rz:rz + nz, rx:rx + nx] = a          # ext[p][q][s] = ã[p-ry][q-rz][s-rx]
    out = np.zeros_like(a)
    for l in range(ky):
        for j in range(kz):
            for i in range(kx):
                w = k[l, j, i]
                if w == 0.0:
                    continue
                out += w * ext[2 * ry - l: 2 * ry - l + ny, 2 * rz - j: 2 * rz - j + nz,
                               2 * rx - i: 2 * rx - i + nx]
    return out


def conv3d_fft(a, k) -> np.ndarray:
    """The same zero-extended convolution through scipy's FFT convolution
    (its centred ``same`` crop of the full linear convolution), for PSFs too
    large for the direct sum."""
    return scipy.signal.fftconvolve(np.asarray(a, dtype=np.float64), np.asarray(k, dtype=np.float64),
                                    mode="same")


def flip3(k) -> np.ndarray:
    return np.asarray(k, dtype=np.float64)[::-1, ::-1, ::-1].copy()


def gaussian_psf3(k: int, sy: float, sx: float, sz: float, ky: int | None = None) -> np.ndarray:
    """Normalised point-sampled 3D Gaussian ``[ky][k][k]`` (y extent ky, default k)."""
    ky = k if ky is None else ky
    y = np.arange(ky) - (ky - 1) / 2
    z = np.arange(k) - (k - 1) / 2
    x = np.arange(k) - (k - 1) / 2
    gy = np.exp(-0.5 * (y / sy) ** 2) if sy > 0 else (y == 0).astype(np.float64)
    g = gy[:, None, None] * np.exp(-0.5 * (z / sz) ** 2)[None, :, None] * np.exp(-0.5 * (x / sx) ** 2)[None, None, :]
    return g / g.sum()


def rl3d_iteration(psi, phis, psfs3, method: str = "direct"):
    """ψ · Π_v [(φ_v / (ψ ⊛ P_v)) ⊛ P_v^*] with 3D kernels (simultaneous update)."""
    conv = conv3d_fft if method == "fft" else conv3d
    prod = np.ones_like(psi)
    for phi, p in zip(phis, psfs3):
        b = conv(psi, p)
        prod = prod * conv(ratio(phi, b), flip3(p))
    return psi * prod


def deconvolve3d(phis, psfs3, iters: int, method: str = "direct") -> np.ndarray:
    """Full 3D MV-RL from the mean of the views, planes ``[Y][Z][X]`` in and out."""
    phis = [np.asarray(p, dtype=np.float64) for p in phis]
    psi = sum(phis) / len(phis)
    for _ in range(int(iters)):
        psi = rl3d_iteration(psi, phis, psfs3, method)
    return psi


__all__ = ["conv3d", "conv3d_fft", "flip3", "gaussian_psf3", "rl3d_iteration", "deconvolve3d", "EPS"]
