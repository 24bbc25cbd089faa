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
import os
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "gaussian_psf",
    "nucleus",
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
    # Planes of the 2048³ size class: 2 views, 64 planes of 2048×2048 (planes
    # are independent, so a slab times the per-plane rate of the full volume).
    "planes2048": VolumeSpec("planes2048", 64, 2048, 2048, 31, (1.5, 6.0), (0, 90),
                             (64 * 2048 * 2048) // (16 ** 3), "u16", 10, "simultaneous", seed=6),
    # The whole 2048³ size class: 2 views, 2048 planes of 2048×2048, 31×31, uint16.
    # (Rendering every plane on the host is slow; the benchmark renders a slab
    # of distinct planes and repeats it along the plane axis on the device.)
    "vol2048": VolumeSpec("vol2048", 2048, 2048, 2048, 31, (1.5, 6.0), (0, 90),
                          (2048 ** 3) // (16 ** 3), "u16", 10, "simultaneous", seed=7),
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


_CHUNK = 16   # planes per generation chunk (noise seeds are per chunk, so results
              # do not depend on how many worker processes are used)


def _render_chunk(args):
    shape_zyx, blobs, y0, y1, background, sig, noise, dtype, seed_key = args
    nz, _, nx = shape_zyx
    sel = (blobs.cy + 4 * np.sqrt(blobs.sigma ** 2) + 1 >= y0) & (blobs.cy - 4 * blobs.sigma - 1 < y1)
    sub = Blobs(cy=blobs.cy[sel] - y0, cz=blobs.cz[sel], cx=blobs.cx[sel], sigma=blobs.sigma[sel],
                amp=blobs.amp[sel])
    lam = render((nz, y1 - y0, nx), sub, background, sig[0], sig[1])
    if not noise:
        return lam
    rng = np.random.default_rng(np.random.SeedSequence(list(seed_key)))
    counts = rng.poisson(lam)
    if dtype == "u16":
        return np.minimum(counts, 65535).astype(np.uint16)
    return counts.astype(np.float32)


def _spawn_safe() -> bool:
    """Spawned workers re-import ``__main__``; that needs a real file."""
    import sys

    main = sys.modules.get("__main__")
    f = getattr(main, "__file__", None)
    return bool(f) and os.path.exists(f)


def _render_volume(shape_zyx, blobs, background, sig, noise, dtype, seed_key, workers):
    ny = shape_zyx[1]
    jobs = [(shape_zyx, blobs, y0, min(ny, y0 + _CHUNK), background, sig, noise, dtype,
             (*seed_key, y0 // _CHUNK)) for y0 in range(0, ny, _CHUNK)]
    if workers > 1 and len(jobs) > 1 and _spawn_safe():
        import concurrent.futures as cf
        import multiprocessing as mp

        with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
            parts = list(ex.map(_render_chunk, jobs))
    else:
        parts = [_render_chunk(j) for j in jobs]
    return np.concatenate(parts, axis=1) if len(parts) > 1 else parts[0]


def make_volume(spec: VolumeSpec, seed: int | None = None, noise: bool = True,
                planes: int | None = None, truth: bool = True, workers: int | None = None):
    """Draw truth and per-view observations for ``spec``.

    Returns ``dict(truth=[Z][Y][X] float32 or None, stacks=[V × [Z][Y][X]],
    psfs=[V × K×K float32])``.  Stacks are uint16 (clipped to 65535) for
    ``obs_dtype == "u16"``, float32 otherwise.  ``noise=False`` returns the
    noise-free blurred intensities (float32).  ``planes`` overrides the number
    of planes Y (reduced volumes with the same plane shape and blob density).
    Large volumes are rendered by ``workers`` processes in chunks of planes;
    the result does not depend on the worker count.
    """
    seed = spec.seed if seed is None else seed
    ny = spec.n_planes if planes is None else int(planes)
    shape = (spec.n_z, ny, spec.n_x)
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0]))
    n_blobs = spec.n_blobs
    if planes is not None and planes != spec.n_planes:
        n_blobs = max(1, int(round(spec.n_blobs * ny / spec.n_planes)))
    blobs = draw_blobs(rng, shape, n_blobs)
    if workers is None:
        big = spec.n_z * ny * spec.n_x > (1 << 24)
        workers = min(8, os.cpu_count() or 1) if big else 1
    tr = None
    if truth:
        tr = _render_volume(shape, blobs, spec.background, (0.0, 0.0), False, "f32", (seed, 0), workers)
    stacks = []
    for v, sig in enumerate(spec.view_sigmas()):
        stacks.append(_render_volume(shape, blobs, spec.background, sig, noise, spec.obs_dtype,
                                     (seed, v + 1), workers))
    return dict(truth=tr, stacks=stacks, psfs=spec.psfs(), blobs=blobs)


def nucleus(shape_yzx, seed: int, radii=(12.0, 14.0, 16.0), n_spots: int = 120, background: float = 10.0,
            amplitude: float = 300.0) -> np.ndarray:
    """One simulated nucleus in planes order ``[Y][Z][X]`` (float64): a
    soft-edged ellipsoid (semi-axes ``radii`` along y, z, x, centred) whose
    interior carries chromatin-like texture, a sum of ``n_spots`` Gaussian
    spots (σ ~ U[1, 2] px, weight ~ U[0.5, 1]) at uniform positions inside
    80% of the semi-axes; intensity background + amplitude · body ·
    (0.4 + texture / max texture)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 7]))
    ny, nz, nx = shape_yzx
    c = np.array([ny / 2, nz / 2, nx / 2])
    rad = np.asarray(radii, dtype=np.float64)
    yy, zz, xx = np.meshgrid(np.arange(ny), np.arange(nz), np.arange(nx), indexing="ij")
    d = np.sqrt(((yy - c[0]) / rad[0]) ** 2 + ((zz - c[1]) / rad[1]) ** 2 + ((xx - c[2]) / rad[2]) ** 2)
    body = 1.0 / (1.0 + np.exp((d - 1.0) * 12.0))
    tex = np.zeros(shape_yzx)
    for _ in range(n_spots):
        p = c + (rng.random(3) * 2 - 1) * rad * 0.8
        sd = rng.uniform(1.0, 2.0)
        tex += rng.uniform(0.5, 1.0) * np.exp(-((yy - p[0]) ** 2 + (zz - p[1]) ** 2 + (xx - p[2]) ** 2) / (2 * sd * sd))
    return background + amplitude * body * (0.4 + tex / tex.max())


def render_planes(spec: VolumeSpec, planes, seed: int | None = None, noise: bool = True):
    """Observations of only the listed planes of ``spec``'s full volume (same
    blob draw as ``make_volume``), for checks at full size that need a few real
    planes only.  Noise is drawn per plane, so the values differ from the
    chunked ``make_volume`` draw.  Returns ``[V × [Z][len(planes)][X]]``."""
    seed = spec.seed if seed is None else seed
    shape = (spec.n_z, spec.n_planes, spec.n_x)
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0]))
    blobs = draw_blobs(rng, shape, spec.n_blobs)
    out = []
    for v, sig in enumerate(spec.view_sigmas()):
        parts = [_render_chunk((shape, blobs, int(y), int(y) + 1, spec.background, sig, noise, spec.obs_dtype,
                                (seed, v + 1, 1 << 20, int(y)))) for y in planes]
        out.append(np.concatenate(parts, axis=1))
    return out
