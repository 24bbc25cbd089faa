"""Seeded synthetic inputs for plane-wise multi-view deconvolution.

This module only makes inputs: blob-nuclei volumes, per-view observations and
Gaussian PSF taps.  It holds none of the deconvolution arithmetic (no discrete
convolution, no Richardson-Lucy step), so the oracle and the GPU path can both
take their inputs from here without sharing any of the method.

Observations are blurred *analytically*: every blob is an isotropic 3D Gaussian,
and the blur of a Gaussian by a Gaussian PSF is again a Gaussian whose variance
is the sum of the two (per axis), with the amplitude scaled so that the blob's
integral is kept.  The 2D view PSF of the plane-wise model acts in the plane
orthogonal to the rotation axis (the Z and X axes here; the rotation axis is Y,
the camera row axis), so only the Z and X widths grow.  Poisson noise is then
drawn per voxel, the noise model of photon counts.

Volumes are returned camera-ordered, ``[Z][Y][X]`` (Z = stack slice, Y = camera
row = rotation axis, X = camera column), which is what the reslice turns into
planes ``[Y][Z][X]``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "gaussian_psf",
    "Blobs",
    "draw_blobs",
    "render",
    "VolumeSpec",
    "CONFIGS",
    "make_volume",
    "random_psf",
]


def gaussian_psf(k: int, sigma_x: float, sigma_z: float, kz: int | None = None) -> np.ndarray:
    """Point-sampled anisotropic 2D Gaussian, normalised to unit sum in FP64.

    Rows are Z offsets, columns X offsets: ``p[j][i] ∝ exp(-dx²/2σx² - dz²/2σz²)``
    with ``dx = i - (kx-1)/2`` and ``dz = j - (kz-1)/2``.  Returned as float64;
    callers cast to float32 for the library.
    """
    kx = int(k)
    kz = int(k if kz is None else kz)
    if kx < 1 or kz < 1 or kx % 2 == 0 or kz % 2 == 0:
        raise ValueError("PSF sides must be odd and >= 1")
    dx = np.arange(kx, dtype=np.float64) - (kx - 1) / 2.0
    dz = np.arange(kz, dtype=np.float64) - (kz - 1) / 2.0
    gx = np.exp(-(dx * dx) / (2.0 * sigma_x * sigma_x))
    gz = np.exp(-(dz * dz) / (2.0 * sigma_z * sigma_z))
    p = np.outer(gz, gx)
    return p / p.sum()


def random_psf(rng: np.random.Generator, kz: int, kx: int, separable: bool = False) -> np.ndarray:
    """Random non-negative, asymmetric PSF (unit sum, FP64) for tests.

    Asymmetric taps make a missing or doubled flip visible.  ``separable``
    returns an outer product of two random positive vectors (rank one).
    """
    if separable:
        p = np.outer(rng.uniform(0.05, 1.0, kz), rng.uniform(0.05, 1.0, kx))
    else:
        p = rng.uniform(0.0, 1.0, (kz, kx))
        p[(kz - 1) // 2, (kx - 1) // 2] += 1.0
    return p / p.sum()


@dataclass
class Blobs:
    """Isotropic Gaussian blobs: centres (y, z, x), widths and amplitudes."""

    cy: np.ndarray
    cz: np.ndarray
    cx: np.ndarray
    sigma: np.ndarray
    amp: np.ndarray


def draw_blobs(rng: np.random.Generator, shape_zyx, n: int,
               sigma=(2.0, 4.0), amp=(200.0, 1000.0)) -> Blobs:
    """Uniform centres inside the volume, σ ~ U[σ0, σ1], amplitude ~ U[a0, a1]."""
    nz, ny, nx = shape_zyx
    cz = rng.uniform(0, nz, n)
    cy = rng.uniform(0, ny, n)
    cx = rng.uniform(0, nx, n)
    s = rng.uniform(sigma[0], sigma[1], n)
    a = rng.uniform(amp[0], amp[1], n)
    return Blobs(cy=cy, cz=cz, cx=cx, sigma=s, amp=a)


def _axis_profile(c: float, s: float, n: int, half: int):
    lo = max(0, int(math.floor(c - half)))
    hi = min(n, int(math.ceil(c + half)) + 1)
    if hi <= lo:
        return lo, hi, None
    d = np.arange(lo, hi, dtype=np.float64) - c
    return lo, hi, np.exp(-(d * d) / (2.0 * s * s))


def render(shape_zyx, blobs: Blobs, background: float,
           psf_sigma_x: float = 0.0, psf_sigma_z: float = 0.0,
           dtype=np.float32) -> np.ndarray:
    """Render ``background + Σ blobs`` into a camera-ordered ``[Z][Y][X]`` volume.

    With ``psf_sigma_x/z > 0`` each blob is rendered already blurred by a
    continuous Gaussian of those widths along X and Z (variances add, the
    amplitude is scaled by ``σ_b/s_x · σ_b/s_z`` so the integral is kept).
    Each blob is evaluated in a box of ±4 widths per axis.
    """
    nz, ny, nx = shape_zyx
    vol = np.full(shape_zyx, background, dtype=dtype)
    for cy, cz, cx, s, a in zip(blobs.cy, blobs.cz, blobs.cx, blobs.sigma, blobs.amp):
        sx = math.sqrt(s * s + psf_sigma_x * psf_sigma_x)
        sz = math.sqrt(s * s + psf_sigma_z * psf_sigma_z)
        scale = a * (s / sx) * (s / sz)
        z0, z1, gz = _axis_profile(cz, sz, nz, math.ceil(4 * sz))
        y0, y1, gy = _axis_profile(cy, s, ny, math.ceil(4 * s))
        x0, x1, gx = _axis_profile(cx, sx, nx, math.ceil(4 * sx))
        if gz is None or gy is None or gx is None:
            continue
        box = (scale * gz)[:, None, None] * gy[None, :, None] * gx[None, None, :]
        vol[z0:z1, y0:y1, x0:x1] += box.astype(dtype, copy=False)
    return vol


@dataclass
class VolumeSpec:
    """One synthetic workload: planes Y of Z rows × X columns, V views."""

    name: str
    n_planes: int          # Y (rotation axis, camera rows)
    n_z: int               # Z (stack slices: plane rows)
    n_x: int               # X (camera columns: plane columns)
    psf_k: int
    psf_sigma: tuple       # (σx, σz) of view 0
    angles: tuple          # degrees; 90/270 swap σx and σz, 180 equals 0
    n_blobs: int
    obs_dtype: str         # "f32" or "u16"
    iters: int
    update: str            # "simultaneous" or "sequential"
    boundary: str = "zero"
    background: float = 100.0
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n_views(self) -> int:
        return len(self.angles)

    def view_sigmas(self):
        sx, sz = self.psf_sigma
        out = []
        for a in self.angles:
            if int(round(a)) % 180 == 90:
                out.append((sz, sx))
            else:
                out.append((sx, sz))
        return out

    def psfs(self):
        """Per-view float32 taps ``[K][K]`` (rows Z, columns X)."""
        return [gaussian_psf(self.psf_k, sx, sz).astype(np.float32)
                for sx, sz in self.view_sigmas()]

    @property
    def voxels(self) -> int:
        return self.n_planes * self.n_z * self.n_x


def _blob_count(spec_shape, per_voxel_side: int) -> int:
    nz, ny, nx = spec_shape
    return max(1, (nz * ny * nx) // (per_voxel_side ** 3))


CONFIGS = {
    # 2 views, 32 planes of 128×128, 15×15 PSFs, 40 blobs, 10 iterations.
    "small": VolumeSpec("small", 32, 128, 128, 15, (1.2, 4.0), (0, 90), 40, "f32", 10,
                        "simultaneous", seed=1),
    # 2 views, 512³, 31×31 PSFs σx=1.5/σz=6, one blob per 16³ voxels, uint16.
    "vol512": VolumeSpec("vol512", 512, 512, 512, 31, (1.5, 6.0), (0, 90),
                         (512 ** 3) // (16 ** 3), "u16", 10, "simultaneous", seed=2),
    # 4 views 0/90/180/270, 1024³, 41×41 PSFs σx=1.5/σz=8, uint16, sequential.
    "vol1024x4": VolumeSpec("vol1024x4", 1024, 1024, 1024, 41, (1.5, 8.0), (0, 90, 180, 270),
                            (1024 ** 3) // (16 ** 3), "u16", 10, "sequential", seed=3),
    # Batched mix: three uneven volumes.
    "mix_a": VolumeSpec("mix_a", 200, 256, 384, 21, (1.5, 4.0), (0, 90), 4800, "f32", 10,
                        "sequential", seed=41),
    "mix_b": VolumeSpec("mix_b", 300, 512, 768, 31, (1.5, 6.0), (0, 90, 180), 28800, "f32", 10,
                        "sequential", seed=42),
    "mix_c": VolumeSpec("mix_c", 150, 1000, 1000, 41, (1.5, 8.0), (0, 90, 180, 270), 36621,
                        "f32", 10, "sequential", seed=43),
    # Differentiation workload: 2 views, 256³, 31×31, 5 iterations.
    "grad256": VolumeSpec("grad256", 256, 256, 256, 31, (1.5, 6.0), (0, 90), 4096, "f32", 5,
                          "simultaneous", seed=5),
}


def make_volume(spec: VolumeSpec, seed: int | None = None, noise: bool = True,
                planes: int | None = None):
    """Draw truth and per-view observations for ``spec``.

    Returns ``dict(truth=[Z][Y][X] float32, stacks=[V × [Z][Y][X]], psfs=[V × K×K float32])``.
    Stacks are uint16 (clipped to 65535) for ``obs_dtype == "u16"``, float32
    otherwise.  ``noise=False`` returns the noise-free blurred intensities
    (float32).  ``planes`` overrides the number of planes Y (for reduced
    test volumes with the same plane shape and density).
    """
    seed = spec.seed if seed is None else seed
    ny = spec.n_planes if planes is None else int(planes)
    shape = (spec.n_z, ny, spec.n_x)
    ss = np.random.SeedSequence(seed)
    blob_seq, *view_seqs = ss.spawn(1 + spec.n_views)
    rng = np.random.default_rng(blob_seq)
    n_blobs = spec.n_blobs
    if planes is not None and planes != spec.n_planes:
        n_blobs = max(1, int(round(spec.n_blobs * ny / spec.n_planes)))
    blobs = draw_blobs(rng, shape, n_blobs)
    truth = render(shape, blobs, spec.background)
    stacks = []
    for (sx, sz), vs in zip(spec.view_sigmas(), view_seqs):
        lam = render(shape, blobs, spec.background, sx, sz)
        if noise:
            vrng = np.random.default_rng(vs)
            counts = vrng.poisson(lam)
            if spec.obs_dtype == "u16":
                obs = np.minimum(counts, 65535).astype(np.uint16)
            else:
                obs = counts.astype(np.float32)
        else:
            obs = lam.astype(np.float32)
        stacks.append(obs)
    return dict(truth=truth, stacks=stacks, psfs=spec.psfs(), blobs=blobs)
