"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these checks re-types the oracle's own formulas: convolution is pinned
to scipy's direct 2D convolution and to the convolution theorem, the whole RL
step to a dense-matrix formulation (A_v built column by column by scipy, the
back-projection taken as the matrix transpose), and the iteration to its
invariants (fixed point of a delta PSF, flux, non-negativity, monotone
I-divergence of EM) and to Gaussian closed forms.
"""
import zlib

import numpy as np
import pytest
import scipy.signal as ss

import oracle
from synthetic import gaussian_psf, random_psf


def _rng(seed=0):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------
# Reslice
# ---------------------------------------------------------------------------
def test_reslice_brute_force_u16():
    st = _rng(1).integers(0, 65536, size=(5, 4, 7), dtype=np.uint16)
    pl = oracle.reslice(st)
    assert pl.shape == (4, 5, 7) and pl.dtype == np.float64
    for z in range(5):
        for y in range(4):
            for x in range(7):
                assert pl[y, z, x] == float(int(st[z, y, x]))


def test_reslice_float_clamps_negative_and_nan():
    st = np.array([[[1.5, -2.0, np.nan]]], dtype=np.float32)  # Z=1, Y=1, X=3
    pl = oracle.reslice(st)
    assert pl.tolist() == [[[1.5, 0.0, 0.0]]]


# ---------------------------------------------------------------------------
# Convolution: library special case, convolution theorem, adjoint identity
# ---------------------------------------------------------------------------
KERNEL_SHAPES = [(1, 1), (3, 3), (5, 3), (3, 7), (9, 9), (15, 15), (11, 13), (1, 9), (9, 1)]
PLANE_SHAPES = [(8, 8), (8, 5), (1, 9), (9, 1), (13, 6)]


@pytest.mark.parametrize("kshape", KERNEL_SHAPES)
@pytest.mark.parametrize("pshape", PLANE_SHAPES)
def test_conv_zero_matches_scipy_fill(kshape, pshape):
    rng = _rng(zlib.crc32(repr((kshape, pshape)).encode()))
    a = rng.standard_normal(pshape)
    k = rng.standard_normal(kshape)
    ref = ss.convolve2d(a, k, mode="same", boundary="fill", fillvalue=0)
    np.testing.assert_allclose(oracle.conv2d(a, k, "zero"), ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kshape", KERNEL_SHAPES)
@pytest.mark.parametrize("pshape", PLANE_SHAPES)
def test_conv_periodic_matches_convolution_theorem(kshape, pshape):
    """Circular convolution via numpy's FFT (kernel centre wrapped to index 0)."""
    rng = _rng(7 + zlib.crc32(repr((kshape, pshape)).encode()))
    a = rng.standard_normal(pshape)
    k = rng.standard_normal(kshape)
    nz, nx = pshape
    kw = np.zeros(pshape)
    rz, rx = (kshape[0] - 1) // 2, (kshape[1] - 1) // 2
    for j in range(kshape[0]):
        for i in range(kshape[1]):
            kw[(j - rz) % nz, (i - rx) % nx] += k[j, i]
    ref = np.real(np.fft.ifft2(np.fft.fft2(a) * np.fft.fft2(kw)))
    np.testing.assert_allclose(oracle.conv2d(a, k, "periodic"), ref, rtol=0, atol=1e-10)
    # scipy's wrap boundary agrees as well
    ref2 = ss.convolve2d(a, k, mode="same", boundary="wrap")
    np.testing.assert_allclose(oracle.conv2d(a, k, "periodic"), ref2, rtol=0, atol=1e-12)


def test_conv_centre_and_orientation_on_impulse():
    """An impulse at (z0, x0) reproduces the kernel with its centre tap at (z0, x0)."""
    a = np.zeros((9, 11))
    a[4, 5] = 1.0
    k = np.arange(15, dtype=np.float64).reshape(3, 5)     # asymmetric
    out = oracle.conv2d(a, k, "zero")
    np.testing.assert_array_equal(out[3:6, 3:8], k)
    out = oracle.conv2d(a, oracle.flip(k), "zero")
    np.testing.assert_array_equal(out[3:6, 3:8], k[::-1, ::-1])


@pytest.mark.parametrize("boundary", ["zero", "periodic"])
@pytest.mark.parametrize("kshape", [(3, 5), (7, 7), (11, 13)])
def test_conv_adjoint_identity(boundary, kshape):
    """⟨a ⊛ k, b⟩ = ⟨a, b ⊛ flip(k)⟩: the flipped PSF is the adjoint operator."""
    rng = _rng(3)
    a = rng.standard_normal((9, 8))
    b = rng.standard_normal((9, 8))
    k = rng.standard_normal(kshape)
    lhs = np.sum(oracle.conv2d(a, k, boundary) * b)
    rhs = np.sum(a * oracle.conv2d(b, oracle.flip(k), boundary))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_conv_fft_method_matches_direct(boundary):
    rng = _rng(5)
    a = rng.random((3, 40, 33))
    for kshape in [(1, 1), (7, 5), (31, 31), (45, 9)]:
        k = rng.random(kshape)
        d = oracle.conv2d(a, k, boundary)
        f = oracle.conv2d(a, k, boundary, method="fft")
        np.testing.assert_allclose(f, d, rtol=0, atol=1e-12 * np.abs(d).max())


def test_conv_batched_over_planes():
    rng = _rng(11)
    a = rng.random((4, 10, 12))
    k = rng.random((5, 7))
    out = oracle.conv2d(a, k, "zero")
    for y in range(4):
        ref = ss.convolve2d(a[y], k, mode="same", boundary="fill")
        np.testing.assert_allclose(out[y], ref, atol=1e-13)


# ---------------------------------------------------------------------------
# Whole RL step vs a dense-matrix formulation
# ---------------------------------------------------------------------------
def _matrix(k, shape, boundary):
    """Dense operator of 'same' convolution, built column by column with scipy."""
    n = shape[0] * shape[1]
    m = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        e = e.reshape(shape)
        bd = "fill" if boundary == "zero" else "wrap"
        m[:, c] = ss.convolve2d(e, k, mode="same", boundary=bd).ravel()
    return m


def _dense_step(psi, phis, mats, backs, ws, update, normalize=False):
    def factor(cur, phi, a, b, w):
        d = a @ cur
        r = np.where(d > oracle.EPS, phi / np.where(d > oracle.EPS, d, 1.0), 1.0)
        q = b @ r
        if normalize:                       # EM form: divide by the column sums b·1
            q = q / (b @ np.ones_like(r))
        return w * q + (1.0 - w)

    if update == "simultaneous":
        prod = np.ones_like(psi)
        for phi, a, b, w in zip(phis, mats, backs, ws):
            prod = prod * factor(psi, phi, a, b, w)
        return psi * prod
    cur = psi
    for phi, a, b, w in zip(phis, mats, backs, ws):
        cur = cur * factor(cur, phi, a, b, w)
    return cur


@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
@pytest.mark.parametrize("nv", [1, 2, 3])
def test_rl_step_matches_dense_matrix_form(update, boundary, nv):
    rng = _rng(100 + nv)
    shape = (8, 8)
    psfs = [random_psf(rng, kz, kx) for kz, kx in [(5, 3), (3, 7), (9, 9)][:nv]]
    phis = [rng.uniform(0.0, 50.0, shape) for _ in range(nv)]
    psi0 = rng.uniform(1.0, 10.0, shape)
    ws = [1.0, 0.7, 0.35][:nv]
    mats = [_matrix(p, shape, boundary) for p in psfs]
    backs_t = [m.T for m in mats]                         # Independent: X = P^*
    ref = _dense_step(psi0.ravel(), [p.ravel() for p in phis], mats, backs_t, ws, update)
    backs = [oracle.back_projector(psfs, v) for v in range(nv)]
    got = oracle.rl_iteration(psi0, phis, psfs, backs, ws, update, boundary)
    np.testing.assert_allclose(got.ravel(), ref, rtol=1e-12, atol=1e-12)

    # an explicit, unrelated back-projector is applied as a plain convolution
    xs = [random_psf(rng, 3, 5) for _ in range(nv)]
    bm = [_matrix(x, shape, boundary) for x in xs]
    ref = _dense_step(psi0.ravel(), [p.ravel() for p in phis], mats, bm, ws, update)
    got = oracle.rl_iteration(psi0, phis, psfs, xs, ws, update, boundary)
    np.testing.assert_allclose(got.ravel(), ref, rtol=1e-12, atol=1e-12)


def test_division_guard_matches_dense_form():
    """Where ψ ⊛ P ≤ ε the ratio is 1; the dense form with the same convention agrees."""
    rng = _rng(9)
    shape = (8, 8)
    psf = random_psf(rng, 3, 3)
    phi = rng.uniform(1.0, 5.0, shape)
    psi0 = rng.uniform(1.0, 5.0, shape)
    psi0[:, :5] = 0.0          # blurred estimate is exactly 0 in columns 0..3
    m = _matrix(psf, shape, "zero")
    ref = _dense_step(psi0.ravel(), [phi.ravel()], [m], [m.T], [1.0], "simultaneous")
    got = oracle.rl_iteration(psi0, [phi], [psf], [oracle.flip(psf)])
    assert np.all(np.isfinite(got))
    np.testing.assert_allclose(got.ravel(), ref, rtol=1e-12, atol=1e-12)
    b = oracle.conv2d(psi0, psf)
    r = oracle.ratio(phi, b)
    assert np.all(r[:, :4] == 1.0)


def test_textbook_richardson_lucy_single_view():
    """V=1, X=P^*, constant start: classic Richardson-Lucy with scipy convolutions."""
    rng = _rng(21)
    shape = (12, 10)
    psf = random_psf(rng, 5, 3)
    phi = rng.uniform(0.0, 30.0, shape)
    u = np.full(shape, 2.0)
    for _ in range(5):
        est = ss.convolve2d(u, psf, mode="same")
        u = u * ss.convolve2d(phi / est, psf[::-1, ::-1], mode="same")
    got = oracle.deconvolve([phi[None]], [psf], 5, init="const", init_const=2.0,
                            layout="planes_yzx")[0]
    np.testing.assert_allclose(got, u, rtol=1e-11)


# ---------------------------------------------------------------------------
# Invariants of the iteration
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
@pytest.mark.parametrize("nv", [1, 2, 4])
def test_delta_psf_is_a_fixed_point(update, nv):
    rng = _rng(31)
    phi = rng.uniform(0.0, 100.0, (3, 9, 7))
    delta = np.ones((1, 1))
    out = oracle.deconvolve([phi] * nv, [delta] * nv, 6, update=update, layout="planes_yzx")
    np.testing.assert_array_equal(out, phi)
    # a zero-padded delta of larger size behaves the same
    d5 = np.zeros((5, 3))
    d5[2, 1] = 1.0
    out = oracle.deconvolve([phi] * nv, [d5] * nv, 3, update=update, layout="planes_yzx")
    np.testing.assert_allclose(out, phi, rtol=1e-15)


def test_delta_psf_single_view_reaches_data_in_one_step():
    rng = _rng(32)
    phi = rng.uniform(1.0, 100.0, (2, 6, 6))
    out = oracle.deconvolve([phi], [np.ones((1, 1))], 1, init="const", init_const=3.0,
                            layout="planes_yzx")
    np.testing.assert_allclose(out, phi, rtol=1e-15)


@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_flux_single_view_equals_data_flux(boundary):
    rng = _rng(41)
    phi = rng.uniform(0.0, 80.0, (2, 11, 9))
    psf = random_psf(rng, 5, 7) * 0.8       # any non-negative taps, not normalised
    _, hist = oracle.deconvolve([phi], [psf], 4, boundary=boundary, layout="planes_yzx",
                                return_history=True)
    for t in range(1, 5):
        for y in range(2):
            assert abs(hist[t][y].sum() - phi[y].sum()) <= 1e-11 * phi[y].sum()


def test_flux_weighted_single_view():
    rng = _rng(42)
    phi = rng.uniform(0.0, 80.0, (1, 10, 10))
    psf = random_psf(rng, 3, 5)
    psi0 = rng.uniform(5.0, 10.0, phi.shape)
    w = 0.3
    out = oracle.deconvolve([phi], [psf], 1, weights=[w], init="given", init_given=psi0,
                            layout="planes_yzx")
    assert abs(out.sum() - ((1 - w) * psi0.sum() + w * phi.sum())) <= 1e-11 * phi.sum()


def test_flux_sequential_follows_last_view():
    rng = _rng(43)
    phis = [rng.uniform(0.0, 80.0, (1, 10, 10)) for _ in range(3)]
    psfs = [random_psf(rng, 3, 5), random_psf(rng, 5, 3), random_psf(rng, 3, 3)]
    out = oracle.deconvolve(phis, psfs, 2, update="sequential", layout="planes_yzx")
    assert abs(out.sum() - phis[-1].sum()) <= 1e-11 * phis[-1].sum()


@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_non_negative(update, boundary):
    rng = _rng(51)
    phis = [rng.uniform(0.0, 50.0, (2, 12, 12)) * (rng.random((2, 12, 12)) > 0.3)
            for _ in range(3)]
    psfs = [random_psf(rng, 5, 5) * (rng.random((5, 5)) > 0.3) for _ in range(3)]
    for p in psfs:
        p[2, 2] = 0.5
    out = oracle.deconvolve(phis, psfs, 5, update=update, boundary=boundary,
                            weights=[1.0, 0.5, 0.0], layout="planes_yzx")
    assert np.all(out >= 0.0) and np.all(np.isfinite(out))


def _noise_free_pair(nv_angles, shape=(1, 48, 48), k=15, sig=(1.2, 4.0), seed=61):
    rng = _rng(seed)
    truth = 100.0 + 800.0 * (rng.random(shape) > 0.97)
    psfs = []
    for a in nv_angles:
        sx, sz = sig if a % 180 == 0 else sig[::-1]
        psfs.append(gaussian_psf(k, sx, sz))
    phis = [oracle.conv2d(truth, p, "periodic") for p in psfs]
    return truth, phis, psfs


def test_i_divergence_monotone_single_view_periodic():
    """Plain RL is EM for Poisson data; with Aᵀ1 = 1 the I-divergence never rises."""
    rng = _rng(62)
    phi = rng.poisson(rng.uniform(20.0, 200.0, (1, 32, 32))).astype(np.float64)
    psf = gaussian_psf(9, 1.3, 2.5)
    psi = oracle.init_estimate([phi])
    back = oracle.flip(psf)
    prev = oracle.i_divergence(psi, [phi], [psf], "periodic")
    for _ in range(12):
        psi = oracle.rl_iteration(psi, [phi], [psf], [back], boundary="periodic")
        cur = oracle.i_divergence(psi, [phi], [psf], "periodic")
        assert cur <= prev * (1 + 1e-12)
        prev = cur


@pytest.mark.parametrize("update,angles", [("simultaneous", (0, 90)),
                                           ("sequential", (0, 90)),
                                           ("sequential", (0, 90, 180, 270))])
def test_i_divergence_monotone_noise_free_multi_view(update, angles):
    truth, phis, psfs = _noise_free_pair(angles)
    backs = [oracle.flip(p) for p in psfs]
    psi = oracle.init_estimate(phis)
    prev = oracle.i_divergence(psi, phis, psfs, "periodic")
    for _ in range(10):
        psi = oracle.rl_iteration(psi, phis, psfs, backs, update=update, boundary="periodic")
        cur = oracle.i_divergence(psi, phis, psfs, "periodic")
        assert cur <= prev * (1 + 1e-12)
        prev = cur


def test_simultaneous_form_overshoots_with_four_views():
    """The printed simultaneous product over-relaxes for V ≥ 3: the I-divergence
    grows where the sequential order keeps falling.  Documents the behaviour of
    the update equation so that nobody 'fixes' it silently."""
    truth, phis, psfs = _noise_free_pair((0, 90, 180, 270))
    backs = [oracle.flip(p) for p in psfs]
    d0 = oracle.i_divergence(oracle.init_estimate(phis), phis, psfs, "periodic")
    psi = oracle.init_estimate(phis)
    for _ in range(10):
        psi = oracle.rl_iteration(psi, phis, psfs, backs, update="simultaneous",
                                  boundary="periodic")
    with np.errstate(all="ignore"):
        d_sim = oracle.i_divergence(psi, phis, psfs, "periodic")
    assert not (d_sim < d0)


# ---------------------------------------------------------------------------
# Compound back-projectors: Gaussian closed forms
# ---------------------------------------------------------------------------
def test_opt2_of_gaussian_is_narrower_gaussian():
    """(P^*)^V of a point-sampled Gaussian is the point-sampled Gaussian of σ/√V."""
    p0 = gaussian_psf(21, 1.5, 4.0)
    p1 = gaussian_psf(21, 4.0, 1.5)
    for nv in (2, 3):
        ps = [p0, p1, p0][:nv]
        x = oracle.back_projector(ps, 0, "opt2")
        ref = gaussian_psf(21, 1.5 / np.sqrt(nv), 4.0 / np.sqrt(nv))
        np.testing.assert_allclose(x, ref, rtol=1e-12, atol=1e-300)


def _gauss_precision_form(k, sig_v, var_terms):
    """Gaussian with precisions 1/σ_v² + Σ 1/var (per axis), point-sampled, unit sum."""
    px = 1.0 / sig_v[0] ** 2 + sum(1.0 / t[0] for t in var_terms)
    pz = 1.0 / sig_v[1] ** 2 + sum(1.0 / t[1] for t in var_terms)
    return gaussian_psf(k, 1.0 / np.sqrt(px), 1.0 / np.sqrt(pz))


def test_efficient_bayes_and_opt1_gaussian_closed_forms():
    """Convolving Gaussians adds variances; pixel-wise products add precisions."""
    k = 41
    s0, s1 = (1.5, 4.0), (4.0, 1.5)
    p0, p1 = gaussian_psf(k, *s0), gaussian_psf(k, *s1)
    eb = oracle.back_projector([p0, p1], 0, "efficient_bayes")
    ref = _gauss_precision_form(k, s0, [(s0[0] ** 2 + 2 * s1[0] ** 2, s0[1] ** 2 + 2 * s1[1] ** 2)])
    np.testing.assert_allclose(eb, ref, rtol=0, atol=1e-6 * ref.max())
    o1 = oracle.back_projector([p0, p1], 0, "opt1")
    ref = _gauss_precision_form(k, s0, [(s0[0] ** 2 + s1[0] ** 2, s0[1] ** 2 + s1[1] ** 2)])
    np.testing.assert_allclose(o1, ref, rtol=0, atol=1e-6 * ref.max())


def test_compound_kernels_single_view_reduce_to_flipped_normalised():
    rng = _rng(71)
    p = random_psf(rng, 5, 7) * 3.0
    f = oracle.flip(p)
    for mode in ("efficient_bayes", "opt1", "opt2"):
        np.testing.assert_allclose(oracle.back_projector([p], 0, mode), f / f.sum(), rtol=1e-14)


def test_compound_kernel_uses_flip_of_own_view():
    """With an asymmetric PSF the compound kernel is built from P_v^*, not P_v."""
    rng = _rng(72)
    p0 = random_psf(rng, 5, 5)
    p1 = np.zeros((5, 5))
    p1[2, 2] = 1.0                               # delta partner view
    # EB with a delta partner: P0^* ⊙ C(P0^* ⊛ δ ⊛ δ) = (P0^*)², normalised
    x = oracle.back_projector([p0, p1], 0, "efficient_bayes")
    f = p0[::-1, ::-1]
    np.testing.assert_allclose(x, f * f / (f * f).sum(), rtol=1e-13)


# ---------------------------------------------------------------------------
# EM-normalised back-projection (divide by X ⊛ 1 = Aᵀ1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
@pytest.mark.parametrize("nv", [1, 2, 3])
def test_normalized_step_matches_dense_matrix_form(update, boundary, nv):
    """ψ · Π_v [w · Aᵀ(φ/Aψ) / Aᵀ1 + 1 − w] with A built column by column."""
    rng = _rng(400 + nv)
    shape = (9, 7)
    psfs = [random_psf(rng, kz, kx) for kz, kx in [(5, 3), (3, 7), (9, 9)][:nv]]
    phis = [rng.uniform(0.0, 50.0, shape) for _ in range(nv)]
    psi0 = rng.uniform(1.0, 10.0, shape)
    ws = [1.0, 0.6, 0.3][:nv]
    mats = [_matrix(p, shape, boundary) for p in psfs]
    ref = _dense_step(psi0.ravel(), [p.ravel() for p in phis], mats, [m.T for m in mats], ws, update,
                      normalize=True)
    backs = [oracle.back_projector(psfs, v) for v in range(nv)]
    got = oracle.rl_iteration(psi0, phis, psfs, backs, ws, update, boundary, normalize=True)
    np.testing.assert_allclose(got.ravel(), ref, rtol=1e-12, atol=1e-12)


def test_sensitivity_is_column_sums():
    """1 ⊛ X is Aᵀ1 for X = flip(P): the column sums of the zero-boundary operator,
    below the tap sum only within R of the edges."""
    rng = _rng(410)
    psf = random_psf(rng, 7, 5)
    shape = (11, 13)
    m = _matrix(psf, shape, "zero")
    s = oracle.sensitivity(shape, oracle.flip(psf), "zero")
    np.testing.assert_allclose(s.ravel(), m.sum(axis=0), rtol=1e-13, atol=1e-15)
    inner = s[3:-3, 2:-2]
    np.testing.assert_allclose(inner, psf.sum(), rtol=1e-13)
    assert s[0, 0] < psf.sum()


def test_normalized_flux_identity_zero_boundary():
    """V = 1, w = 1: Σ (Aᵀ1)·ψ' = Σ φ for the normalised update (where Aψ > ε),
    while the unnormalised update misses it under the zero boundary."""
    rng = _rng(411)
    psf = gaussian_psf(9, 1.4, 2.6)
    phi = rng.uniform(20.0, 300.0, (1, 24, 20))
    psi = rng.uniform(50.0, 150.0, (1, 24, 20))
    back = oracle.flip(psf)
    s = oracle.sensitivity((24, 20), back, "zero")
    nxt = oracle.rl_iteration(psi, [phi], [psf], [back], boundary="zero", normalize=True)
    assert abs(float(np.sum(s * nxt)) - float(np.sum(phi))) <= 1e-10 * float(np.sum(phi))
    plain = oracle.rl_iteration(psi, [phi], [psf], [back], boundary="zero")
    assert abs(float(np.sum(s * plain)) - float(np.sum(phi))) > 1e-6 * float(np.sum(phi))


def test_normalized_i_divergence_monotone_zero_boundary():
    """The normalised single-view update is EM for Poisson data under the zero
    boundary too, so its I-divergence never rises (plain RL's does rise there)."""
    rng = _rng(412)
    phi = rng.poisson(rng.uniform(20.0, 200.0, (1, 32, 28))).astype(np.float64)
    psf = gaussian_psf(9, 1.3, 2.5)
    back = oracle.flip(psf)
    psi = oracle.init_estimate([phi])
    prev = oracle.i_divergence(psi, [phi], [psf], "zero")
    for _ in range(12):
        psi = oracle.rl_iteration(psi, [phi], [psf], [back], boundary="zero", normalize=True)
        cur = oracle.i_divergence(psi, [phi], [psf], "zero")
        assert cur <= prev * (1 + 1e-12)
        prev = cur


def test_normalized_periodic_is_plain_for_unit_sum_kernels():
    """Under the periodic boundary 1 ⊛ X is the tap sum everywhere: for a
    unit-sum back-projector the normalised update is the plain one."""
    rng = _rng(413)
    psfs = [gaussian_psf(7, 1.2, 2.0), gaussian_psf(7, 2.0, 1.2)]
    phis = [rng.uniform(10.0, 90.0, (2, 12, 10)) for _ in range(2)]
    psi = rng.uniform(10.0, 90.0, (2, 12, 10))
    backs = [oracle.flip(p) for p in psfs]
    a = oracle.rl_iteration(psi, phis, psfs, backs, boundary="periodic", normalize=True)
    b = oracle.rl_iteration(psi, phis, psfs, backs, boundary="periodic")
    np.testing.assert_allclose(a, b, rtol=1e-13)


# ---------------------------------------------------------------------------
# Per-pixel view weights
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("update", ["simultaneous", "sequential"])
@pytest.mark.parametrize("normalize", [False, True])
def test_pixel_weights_match_dense_matrix_form(update, normalize):
    """ψ · Π_v [ω_v ⊙ q_v + 1 − ω_v] with per-pixel ω_v, against the dense form
    with the weights applied element by element."""
    rng = _rng(420)
    shape = (8, 9)
    psfs = [random_psf(rng, 5, 3), random_psf(rng, 3, 7)]
    phis = [rng.uniform(0.0, 50.0, shape) for _ in range(2)]
    psi0 = rng.uniform(1.0, 10.0, shape)
    om = [rng.uniform(0.0, 1.0, shape) for _ in range(2)]
    mats = [_matrix(p, shape, "zero") for p in psfs]

    def factor(cur, phi, a, w):
        d = a @ cur
        r = np.where(d > oracle.EPS, phi / np.where(d > oracle.EPS, d, 1.0), 1.0)
        q = a.T @ r
        if normalize:
            q = q / (a.T @ np.ones_like(r))
        return w * q + (1.0 - w)

    cur = psi0.ravel()
    if update == "simultaneous":
        cur = cur * factor(cur, phis[0].ravel(), mats[0], om[0].ravel()) * \
            factor(cur, phis[1].ravel(), mats[1], om[1].ravel())
    else:
        for v in range(2):
            cur = cur * factor(cur, phis[v].ravel(), mats[v], om[v].ravel())
    backs = [oracle.back_projector(psfs, v) for v in range(2)]
    got = oracle.rl_iteration(psi0, phis, psfs, backs, om, update, "zero", normalize=normalize)
    np.testing.assert_allclose(got.ravel(), cur, rtol=1e-12, atol=1e-12)


def test_constant_pixel_weights_equal_scalar_weights():
    rng = _rng(421)
    psfs = [gaussian_psf(7, 1.2, 2.0), gaussian_psf(7, 2.0, 1.2)]
    phis = [rng.uniform(10.0, 90.0, (2, 12, 10)) for _ in range(2)]
    psi = rng.uniform(10.0, 90.0, (2, 12, 10))
    backs = [oracle.flip(p) for p in psfs]
    a = oracle.rl_iteration(psi, phis, psfs, backs, [0.7, 0.3], "sequential", "zero")
    b = oracle.rl_iteration(psi, phis, psfs, backs, [np.full((2, 12, 10), 0.7), np.full((2, 12, 10), 0.3)],
                            "sequential", "zero")
    np.testing.assert_array_equal(a, b)


def test_zero_pixel_weights_freeze_the_estimate_there():
    """Where every view's ω is 0 the estimate does not move."""
    rng = _rng(422)
    psfs = [gaussian_psf(7, 1.2, 2.0), gaussian_psf(7, 2.0, 1.2)]
    phis = [rng.uniform(10.0, 90.0, (1, 16, 12)) for _ in range(2)]
    psi = rng.uniform(10.0, 90.0, (1, 16, 12))
    om = np.ones((1, 16, 12))
    om[:, 4:9, 3:7] = 0.0
    backs = [oracle.flip(p) for p in psfs]
    nxt = oracle.rl_iteration(psi, phis, psfs, backs, [om, om], "simultaneous", "zero")
    np.testing.assert_array_equal(nxt[:, 4:9, 3:7], psi[:, 4:9, 3:7])
    assert np.abs(nxt - psi).max() > 1e-3
