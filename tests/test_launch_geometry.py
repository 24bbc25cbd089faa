"""Host-side model of the separable kernels' index arithmetic.

For launch geometries the planner actually picks (read back through an
internal export of the library), every global-memory and LDS access the
kernels make is recomputed here and checked against its buffer.  This runs on
the CPU so that a planner or indexing mistake shows up before any kernel runs.
The formulas mirror the kernel source (ring rows, work items, 8-wide row-pass
accesses, LDS rows and pads).
"""
import ctypes

import numpy as np
import pytest

from paper_1503_07998_amd import _native as N
from paper_1503_07998_amd import api

G = 8      # rows per ring step
NX = 8     # row-pass outputs per item
LDS_LIMIT = 160 * 1024
MAX_PLANE_X = 65536   # length of the kernels' static zero row (rows outside the plane)


def plan(ctx, Y, k, boundary, one_ring=False):
    out = (ctypes.c_int * 16)()
    lib = N.lib()
    lib.mvd_internal_sep_plan.restype = ctypes.c_int
    lib.mvd_internal_sep_plan.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int)]
    assert lib.mvd_internal_sep_plan(ctx, Y, -k if one_ring else k, N.BOUNDARY[boundary], out) == 0
    keys = ["bucket", "cols", "threads", "occ", "zseg", "nseg", "x_out", "nstrip", "halo", "ncols",
            "ldsw", "vec", "lds_per_view"]
    return dict(zip(keys, list(out)[:len(keys)]))


def check_geometry(Y, Z, X, k, boundary, views, one_ring=False):
    ctx = api.mvd_create(1, Z, X, N.MVD_DEVICE_NONE)
    try:
        p = plan(ctx, Y, k, boundary, one_ring)
    finally:
        api.mvd_destroy(ctx)
    KB = p["bucket"]
    R = (KB - 1) // 2
    M = G * ((2 * G + KB - 1 + G - 1) // G)
    nt, C = p["threads"], p["cols"]
    assert nt % 64 == 0 and 64 <= nt <= 1024
    if nt > 512:   # only the one-column 4-waves/SIMD kernels take such work-groups
        assert one_ring and C == 1 and p["occ"] == 4 and p["halo"] == 0 and X <= nt
    assert views * p["lds_per_view"] <= LDS_LIMIT
    assert p["zseg"] % G == 0 and p["nseg"] * p["zseg"] >= Z and (p["nseg"] - 1) * p["zseg"] < Z
    assert p["nstrip"] * p["x_out"] >= X and (p["nstrip"] - 1) * p["x_out"] < X
    if p["vec"]:
        assert X % 8 == 0 and p["x_out"] % 8 == 0
    halo = p["halo"] != 0
    if boundary == "periodic":
        assert halo, "periodic runs must use strips with wrapped halo columns"
    ldsw = p["ldsw"]
    assert ldsw % 4 == 0
    plane = Z * X
    NIN4 = (NX + KB - 1 + 3) // 4
    for strip in range(p["nstrip"]):
        xo0 = strip * p["x_out"]
        xout = min(p["x_out"], X - xo0)
        assert xout >= 1
        ncz = xout + 2 * R if halo else xout
        assert ncz <= nt * C, "z-pass columns exceed the threads' columns"
        # z-pass columns: LDS column and source column (valid address always)
        for lc in range(ncz):
            x = xo0 - R + lc if halo else lc
            if boundary == "zero":
                ok = 0 <= x < X
            else:
                ok, x = True, x % X
            gx = x if ok else 0
            assert 0 <= gx < X
            lcol = lc if halo else lc + R
            assert 0 <= lcol < ldsw
        if not halo:
            assert R + X <= ldsw
        # row-pass items: LDS reads and global accesses
        nxb = (xout + NX - 1) // NX
        for xb in range(nxb):
            ox = xb * NX
            assert ox + 4 * NIN4 <= ldsw, "row-pass LDS read past the row"
            nvalid = min(NX, xout - ox)
            width = NX if p["vec"] else nvalid
            assert ox + width <= xout or (p["vec"] and xo0 + ox + NX <= X)
            assert xo0 + ox + width <= X, "row-pass access past the row end"
    for seg in range(p["nseg"]):
        zs = seg * p["zseg"]
        ze = min(zs + p["zseg"], Z)
        ngroups = (ze - zs + G - 1) // G
        # ring rows: every row index (incl. the prefetch of the group after the last) is clamped;
        # a row outside the plane under the zero boundary reads the static zero row at the
        # threads' source columns, which must lie inside it
        max_gx = X - 1
        for m in range(0, (ngroups + 1) * G + KB - 1):
            rr = zs - R + m
            if boundary == "zero":
                if 0 <= rr < Z:
                    assert 0 <= rr * X < plane
                else:
                    assert max_gx < MAX_PLANE_X, "zero-row read past its end"
            else:
                assert 0 <= (rr % Z) < Z
        # clamped item rows; the forward pass reads the observations at
        # y·sy + z·sz + x in the layout they were given in (stack or planes)
        for i in range(ngroups):
            for g in range(G):
                z = zs + i * G + g
                zc = z if z < ze else zs
                assert 0 <= zc < Z
                for sy, sz in ((X, Y * X), (Z * X, X)):
                    assert (Y - 1) * sy + zc * sz + X <= Y * Z * X


SHAPES = [
    (2, 1, 37), (2, 41, 1), (3, 8, 8), (4, 37, 53), (2, 70, 100), (2, 13, 200), (2, 24, 700),
    (2, 16, 1100), (1, 12, 600), (2, 9, 66), (32, 128, 128), (512, 512, 512), (200, 256, 384),
    (300, 512, 768), (150, 1000, 1000), (256, 256, 256), (4, 1024, 1024), (2, 5, 2100),
    (1, 3, 513), (1, 7, 1023), (1, 7, 1025), (3, 33, 511),
]


def test_strip_width_never_exceeds_thread_columns():
    """Strips sized against the threads' columns minus the halo, then rounded
    up to whole items, must still fit (one and two columns per thread)."""
    for X in (1000, 1001, 1017, 1023, 2047, 2100, 3000):
        for k in (1, 3, 9, 15, 21, 41, 63):
            ctx = api.mvd_create(1, 16, X, N.MVD_DEVICE_NONE)
            try:
                for b in ("zero", "periodic"):
                    p = plan(ctx, 2, k, b)
                    if p["halo"]:
                        assert p["x_out"] + 2 * p["halo"] <= p["threads"] * p["cols"], (X, k, b, p)
            finally:
                api.mvd_destroy(ctx)


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{y}x{z}x{x}" for y, z, x in SHAPES])
@pytest.mark.parametrize("k", [1, 5, 9, 15, 21, 31, 41, 63])
def test_separable_launch_geometry_in_bounds(shape, k):
    Y, Z, X = shape
    for boundary in ("zero", "periodic"):
        for views in (1, 2):
            check_geometry(Y, Z, X, k, boundary, views)


def mfma_plan(kz, kx):
    out = (ctypes.c_int * 3)()
    lib = N.lib()
    lib.mvd_internal_mfma_plan.restype = ctypes.c_int
    lib.mvd_internal_mfma_plan.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    assert lib.mvd_internal_mfma_plan(kz, kx, out) == 0
    return out[0], out[1], out[2]


@pytest.mark.parametrize("kz", [1, 3, 9, 15, 31, 41, 63])
def test_matrix_core_general_pass_in_bounds(kz):
    """Every LDS access of the matrix-core K×K pass (work-group tile 32 × 64,
    waves at rows 0/16 and columns 0/32, two 16-column blocks each) lies in the
    staged input tile or the tap rows, and the work-group fits in LDS."""
    MZ, MX = 32, 64
    for kx in range(1, 64, 2):
        nck, tw, lds = mfma_plan(kz, kx)
        assert nck > 0 and 4 * nck >= 16 + kx - 1, (kx, nck)      # steps cover the band
        assert tw % 32 == 2
        th, fl = MZ + kz - 1, 4 * nck + 16
        assert lds == 4 * (th * tw + kz * fl) <= LDS_LIMIT
        lane = np.arange(64)
        n, kk = lane % 16, lane // 16
        for m0 in (0, 16):
            for c0 in (0, 32):
                for c in (0, nck - 1):
                    for j in (0, kz - 1):
                        row = m0 + n + j
                        assert row.max() < th and row.min() >= 0
                        for blk in (0, 16):
                            col = c0 + blk + 4 * c + kk
                            assert col.max() < tw
                        fidx = j * fl + 16 + kk - n + 4 * c
                        assert fidx.min() >= j * fl and fidx.max() < (j + 1) * fl
        # output rows and columns of the accumulators stay in the work-group tile
        for i in range(4):
            assert (16 + 4 * (lane // 16) + i).max() < MZ
        assert (32 + 16 + lane % 16).max() < MX


@pytest.mark.parametrize("shape", [(2, 1, 37), (3, 8, 8), (4, 37, 53), (2, 70, 100), (2, 13, 200), (1, 12, 512),
                                   (32, 128, 128), (512, 512, 512), (256, 256, 256), (3, 33, 511), (2, 41, 1),
                                   (2, 13, 520), (2, 24, 700), (2, 16, 1100), (3, 64, 2048), (1, 7, 1023)],
                         ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("k", [1, 5, 9, 15, 21, 31])
def test_split_view_backward_in_bounds(shape, k):
    """The split-view backward form: 1024-thread work-groups, half the threads
    per view (one ring column each), 16-row groups, both views' buffers in LDS;
    whole rows up to 512 columns, wider rows in strips with halo columns."""
    Y, Z, X = shape
    GS = 16
    ctx = api.mvd_create(1, Z, X, N.MVD_DEVICE_NONE)
    try:
        out = (ctypes.c_int * 16)()
        lib = N.lib()
        lib.mvd_internal_split_plan.restype = ctypes.c_int
        lib.mvd_internal_split_plan.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_int)]
        st = lib.mvd_internal_split_plan(ctx, Y, k, out)
    finally:
        api.mvd_destroy(ctx)
    assert st == 0
    keys = ["bucket", "cols", "threads", "occ", "zseg", "nseg", "x_out", "nstrip", "halo", "ncols", "ldsw", "vec",
            "lds"]
    p = dict(zip(keys, list(out)[:13]))
    KB, nt, ldsw = p["bucket"], p["threads"], p["ldsw"]
    R = (KB - 1) // 2
    half = nt // 2
    halo = p["halo"] != 0
    assert nt <= 1024 and nt % 128 == 0 and p["cols"] == 1 and p["occ"] == 4
    assert p["zseg"] % GS == 0 and p["nseg"] * p["zseg"] >= Z and (p["nseg"] - 1) * p["zseg"] < Z
    assert p["nstrip"] * p["x_out"] >= X and (p["nstrip"] - 1) * p["x_out"] < X
    NK = (KB + 3 + 3) // 4 * 4
    assert p["lds"] == 4 * (2 * 2 * GS * ldsw + 2 * 8 * NK) <= LDS_LIMIT
    if not halo:
        assert p["nstrip"] == 1 and half >= X and R + X <= ldsw
    NIN4 = (NX + KB - 1 + 3) // 4
    for strip in range(p["nstrip"]):
        xo0 = strip * p["x_out"]
        xout = min(p["x_out"], X - xo0)
        ncz = xout + 2 * R if halo else xout
        assert ncz <= half, "each half must hold one ring column per thread"
        for lc in range(ncz):
            x = xo0 - R + lc if halo else lc
            gx = x if 0 <= x < X else 0
            assert 0 <= gx < X
            lcol = lc if halo else lc + R
            assert 0 <= lcol < ldsw
        nxb = (xout + NX - 1) // NX
        for xb in range(nxb):
            ox = xb * NX
            assert ox + 4 * NIN4 <= ldsw, "row-pass LDS read past the row"
            if p["vec"]:
                assert xo0 + ox + NX <= X
    # row-pass LDS rows: (view·16 + g) of buffer (i & 1), g < 16
    assert (2 * GS + GS) * ldsw <= 2 * 2 * GS * ldsw   # view 1, row 15 of buffer 0 within both buffers


# ---------------------------------------------------------------------------
# Matrix-core tap-gradient correlation
# ---------------------------------------------------------------------------
MCZ, MCT = 16, 256


def corr_plan(Y, Z, X, kz, kx):
    out = (ctypes.c_long * 7)()
    lib = N.lib()
    lib.mvd_internal_corr_plan.restype = ctypes.c_int
    lib.mvd_internal_corr_plan.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_long)]
    assert lib.mvd_internal_corr_plan(Y, Z, X, kz, kx, out) == 0
    return dict(zip(["kzp", "kxp", "tw", "zch", "nitems", "nblocks", "lds"], list(out)))


def corr_pitch(tw):
    return tw + 2


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 5, 37), (3, 16, 16), (2, 17, 300), (256, 256, 256),
                                   (1024, 1024, 1024), (3, 40, 513), (1, 70, 2048), (300, 150, 1000)],
                         ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("k", [(1, 1), (3, 9), (15, 15), (31, 31), (41, 17), (63, 63)],
                         ids=lambda k: f"{k[0]}x{k[1]}")
def test_matrix_core_correlation_in_bounds(shape, k):
    """Every LDS access of the matrix-core correlation (the ring of staged ã
    rows, the ḡ rows, 16 × 16 × 4 operand lanes, the 4-wave reduction) and
    every partial it writes lies in its buffer; the tiles of a row cover every
    column x' that meets a tap; the work-group fits in LDS."""
    Y, Z, X = shape
    kz, kx = k
    p = corr_plan(Y, Z, X, kz, kx)
    kzp, kxp, tw, zch = p["kzp"], p["kxp"], p["tw"], p["zch"]
    rz, rx = (kz - 1) // 2, (kx - 1) // 2
    assert kzp % 16 == 0 and kxp % 16 == 0 and kz <= kzp <= 64 and kx <= kxp <= 64
    assert tw % 16 == 0 and 16 <= tw <= 256
    width = X + kx - 1
    ntx, ntz = -(-width // tw), -(-Z // MCZ)
    assert ntx * tw >= width and (ntx - 1) * tw < width
    assert 1 <= zch <= ntz and p["nitems"] == Y * ntx * (-(-ntz // zch))
    assert 1 <= p["nblocks"] <= min(1024, p["nitems"])
    nr, pa, pb = MCZ + kzp - 1, corr_pitch(tw), tw + kxp
    assert pa % 4 == 2 and pa >= tw and nr >= MCZ
    # the 32 lanes of a half-wave (16 rows n, 2 columns kk) read 32 distinct banks
    half = (-(np.arange(16)[:, None]) * pa + np.arange(2)[None, :]) % 32
    assert len(np.unique(half)) == 32
    assert p["lds"] == 4 * max(nr * pa + MCZ * pb, 4 * kzp * kxp) <= LDS_LIMIT
    assert (LDS_LIMIT // p["lds"]) * 256 >= p["nblocks"] or p["nblocks"] <= 256
    lane = np.arange(64)
    n, kk = lane % 16, lane // 16
    for ring0 in range(0, nr):
        for zz in (0, MCZ - 1):
            for jb in range(kzp // 16):
                sl = ring0 + zz + kzp - 1 - n - 16 * jb
                assert sl.min() >= 0 and sl.max() < 2 * nr
                sl = np.where(sl < nr, sl, sl - nr)
                assert sl.min() >= 0 and sl.max() < nr
    for q in (0, tw // 4 - 1):
        assert (4 * q + kk).max() < tw
        for ib in range(kxp // 16):
            assert (kk + n + 16 * ib + 4 * q).max() < pb
    # the staging walk: element e = t + u·MCT of a rows × pitch window, rows mapped to ring slots
    for rows, pitch, ringed in ((nr, pa, True), (MCZ, pa, True), (MCZ, pb, False)):
        e = np.arange(MCT)[:, None] + MCT * np.arange(-(-rows * pitch // MCT) + 8)[None, :]
        r, c = e // pitch, e % pitch
        kept = r < rows
        assert (c < pitch).all() and (r[kept] < rows).all()
        for rs in ((0, nr - MCZ, nr - 1) if ringed else (0,)):
            slot = np.where(rs + r < nr, rs + r, rs + r - nr) if ringed else r
            lim = nr * pa if ringed else MCZ * pb
            assert (slot[kept] >= 0).all() and (slot[kept] * pitch + c[kept] < lim).all()
    # reduction: row 16·jb + 4·kk + r, column 16·ib + n of each wave's block
    for w in (0, 3):
        idx = w * kzp * kxp + (16 * (kzp // 16 - 1) + 4 * kk + 3) * kxp + 16 * (kxp // 16 - 1) + n
        assert idx.max() < 4 * kzp * kxp


@pytest.mark.parametrize("boundary", ["zero", "periodic"])
@pytest.mark.parametrize("shape,k", [((2, 19, 37), (7, 5)), ((1, 33, 300), (15, 31)), ((2, 5, 9), (9, 3)),
                                     ((1, 70, 20), (31, 3))],
                         ids=["19x37", "33x300", "5x9", "70x20"])
@pytest.mark.parametrize("zch", [None, 1, 2, 3])
def test_matrix_core_correlation_tiling_model(shape, k, boundary, zch):
    """The tile decomposition of the matrix-core correlation, replayed in
    numpy with the kernel's ring of ã rows: for each tile the staged ã window
    (A[j][x'] = ã[z + Rz − j][x']) times the staged Toeplitz window of ḡ
    (B[x'][i] = ḡ[z][x' − Rx + i]), summed over rows, tiles and runs, equals
    the direct sum Σ ḡ[y][z][x] · ã[y][z + Rz − j][x + Rx − i] over the plane.
    zch=None takes the planner's run length."""
    Y, Z, X = shape
    kz, kx = k
    p = corr_plan(Y, Z, X, kz, kx)
    kzp, kxp, tw = p["kzp"], p["kxp"], p["tw"]
    ntz = -(-Z // MCZ)
    zch = p["zch"] if zch is None else min(zch, ntz)
    rz, rx = (kz - 1) // 2, (kx - 1) // 2
    rng = np.random.default_rng(3)
    src = rng.standard_normal((Y, Z, X))
    gbar = rng.standard_normal((Y, Z, X))

    def sat(y, z, x):
        if boundary == "periodic":
            return src[y, z % Z, x % X]
        return src[y, z, x] if 0 <= z < Z and 0 <= x < X else 0.0

    direct = np.zeros((kz, kx))
    for j in range(kz):
        for i in range(kx):
            for y in range(Y):
                for z in range(Z):
                    for x in range(X):
                        direct[j, i] += gbar[y, z, x] * sat(y, z + rz - j, x + rx - i)
    xa = rx - kx + 1
    ntx = -(-(X + kx - 1) // tw)
    C = np.zeros((kzp, kxp))
    nr, pb = MCZ + kzp - 1, tw + kxp
    ring = np.full((nr, tw), np.nan)
    for y in range(Y):
        for zc in range(-(-ntz // zch)):
            for tx in range(ntx):
                x0 = xa + tx * tw
                tz0 = zc * zch
                ring0 = 0
                for tz in range(tz0, min(ntz, tz0 + zch)):
                    z0 = tz * MCZ
                    za = z0 + rz - (kzp - 1)
                    rfirst = 0 if tz == tz0 else nr - MCZ
                    rs = ring0 + rfirst
                    for r in range(nr - rfirst):
                        slot = rs + r if rs + r < nr else rs + r - nr
                        ring[slot] = [sat(y, za + rfirst + r, x0 + c) for c in range(tw)]
                    Bs = np.array([[gbar[y, z0 + r, x0 - rx + c] if z0 + r < Z and 0 <= x0 - rx + c < X else 0.0
                                    for c in range(pb)] for r in range(MCZ)])
                    for zz in range(min(MCZ, Z - z0)):
                        rows = []
                        for j in range(kzp):
                            sl = ring0 + zz + kzp - 1 - j
                            rows.append(ring[sl if sl < nr else sl - nr])
                        A = np.array(rows)                                            # [kzp][tw]
                        B = np.array([Bs[zz, c:c + kxp] for c in range(tw)])           # [tw][kxp]
                        assert not np.isnan(A).any()
                        C += A @ B
                    ring0 = ring0 + MCZ if ring0 + MCZ < nr else ring0 + MCZ - nr
    np.testing.assert_allclose(C[:kz, :kx], direct, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("shape", [(2, 24, 600), (1, 12, 1000), (3, 40, 1024), (2, 9, 513), (150, 1000, 1000),
                                   (64, 1024, 1024)], ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("k", [3, 15, 31, 41, 63])
def test_wide_rows_geometry_in_bounds(shape, k):
    """One-ring passes over rows of 513–1024 columns plan one column per thread
    in up to 1024-thread work-groups; every access stays in its buffer (the
    same model as the other plans)."""
    import ctypes

    lib = N.lib()
    lib.mvd_internal_set_tune.argtypes = [ctypes.c_char_p]
    try:
        lib.mvd_internal_set_tune(b"")
        Y, Z, X = shape
        for boundary in ("zero", "periodic"):
            check_geometry(Y, Z, X, k, boundary, 1, one_ring=True)
            check_geometry(Y, Z, X, k, boundary, 2, one_ring=True)
    finally:
        lib.mvd_internal_set_tune(None)


@pytest.mark.parametrize("k", [3, 31, 63])
def test_widest_accepted_plane_geometry_in_bounds(k):
    """The widest plane a context accepts (MVD_MAX_PLANE_X columns): strips with
    halos, and every zero-row read inside the static row."""
    for boundary in ("zero", "periodic"):
        check_geometry(1, 3, MAX_PLANE_X, k, boundary, 1)


# ---------------------------------------------------------------------------
# Fused iteration (forward and backward passes of both views in one launch).
# ---------------------------------------------------------------------------
FUSED_BUCKETS = [3, 7, 11, 15, 21, 31]


def fused_plan(ctx, kb):
    out = (ctypes.c_int * 8)()
    lib = N.lib()
    lib.mvd_internal_fused_plan.restype = ctypes.c_int
    lib.mvd_internal_fused_plan.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    assert lib.mvd_internal_fused_plan(ctx, kb, out) == 0
    keys = ["kb", "x_out", "nstrip", "R", "RA", "pitch", "lds", "threads"]
    return dict(zip(keys, list(out)))


def check_fused(Z, X, kb):
    """Every access of the fused kernel for a Z × X plane, bucket kb."""
    ctx = api.mvd_create(2, Z, X, N.MVD_DEVICE_NONE)
    try:
        p = fused_plan(ctx, kb)
    finally:
        api.mvd_destroy(ctx)
    R, RA, pitch, x_out, T = p["R"], p["RA"], p["pitch"], p["x_out"], p["threads"]
    assert R == (kb - 1) // 2 and RA % NX == 0 and RA >= R
    role = T // 3
    assert role % 64 == 0 and T <= 1024
    NK = (kb + 3 + 3) // 4 * 4
    NIN4 = (NX + kb - 1 + 3) // 4
    M = G * ((2 * G + kb - 1 + G - 1) // G)
    U = M // G
    D = (G + R + G - 1) // G
    assert D * G >= G + R
    # LDS: three [2][G][pitch] buffers and two [2][8][NK] tap tables
    setf = 2 * G * pitch
    assert p["lds"] == 4 * (3 * setf + 2 * 2 * 8 * NK) <= LDS_LIMIT
    assert pitch % 8 == 4
    wf, wb = x_out + 2 * RA + 2 * R, x_out + 2 * R
    assert wf <= role and wb <= role          # one column per ring thread
    assert p["nstrip"] == -(-X // x_out)
    # forward row-pass items: threads [0, nfi), view-major, pairs of rows
    nxbF = (x_out + 2 * RA) // NX
    nfi = 2 * G * nxbF
    assert nfi <= 2 * role
    for it in range(nfi):
        v = it // (G * nxbF)
        rem = it - v * G * nxbF
        pr = rem >> 1
        gp = pr // nxbF
        g, ox = 2 * gp + (rem & 1), (pr - gp * nxbF) * NX
        assert 0 <= v < 2 and 0 <= g < G
        assert ox + 4 * NIN4 <= pitch            # bufF reads (columns ≥ wf are zeroed pads)
        assert ox + NX <= x_out + 2 * RA         # bufT writes inside the transferred range
    # backward row-pass items: threads [2·role, 2·role + nbi)
    nxbB = x_out // NX
    nbi = G * nxbB
    assert nbi <= role and nbi % 64 == 0
    for it in range(nbi):
        pr = it >> 1
        gp = pr // nxbB
        g, ox = 2 * gp + (it & 1), (pr - gp * nxbB) * NX
        assert 0 <= g < G and ox + 4 * NIN4 <= pitch
    # transfer into the r rings: role-B thread tr < wb reads bufT column tr + RA − R
    assert 0 <= RA - R and wb - 1 + RA - R < x_out + 2 * RA
    # global accesses per strip: 8-column items lie wholly inside or outside the plane
    assert X % NX == 0
    for s in range(p["nstrip"]):
        x0 = s * x_out
        for ox in range(0, x_out + 2 * RA, NX):
            fx = x0 - RA + ox
            if 0 <= fx < X:
                assert fx + NX <= X
        for ox in range(0, x_out, NX):
            if x0 + ox < X:
                assert x0 + ox + NX <= X
    # ring slots over every phase: the forward ring (ψ rows) and the r rings
    ngroups = -(-Z // G)
    nphases = ngroups + D
    fslot = [None] * M
    for m in range(G + kb - 1):
        fslot[m] = -R + m
    rslot = [None] * M
    for m in range(R):
        rslot[m] = m - R                         # r rows above the plane (zero)
    for ph in range(nphases):
        u = ph % U
        if ph < ngroups:
            for g in range(G):                   # prefetch first, then the column pass
                fslot[((u + 1) * G + kb - 1 + g) % M] = -R + (ph + 1) * G + kb - 1 + g
            for b in range(G // 4):
                for k in range(kb + 3):
                    assert fslot[(u * G + 4 * b + k) % M] == ph * G + 4 * b + k - R
        j = ph - D
        if j >= 0:
            ub = ((u - D) % U + U) % U
            for b in range(G // 4):
                for k in range(kb + 3):
                    assert rslot[(ub * G + 4 * b + k) % M] == j * G + 4 * b + k - R, (ph, b, k)
        for g in range(G):                       # group ph's r rows join the rings
            rslot[(u * G + g + R) % M] = ph * G + g
    # every output row group was back-projected
    assert nphases - D == ngroups


@pytest.mark.parametrize("kb", FUSED_BUCKETS)
@pytest.mark.parametrize("Z,X", [(512, 512), (37, 264), (8, 64), (2048, 2048), (100, 8), (13, 520)])
def test_fused_geometry(Z, X, kb):
    check_fused(Z, X, kb)


def test_fused_plan_rejects_wide_kernels():
    ctx = api.mvd_create(2, 64, 64, N.MVD_DEVICE_NONE)
    try:
        out = (ctypes.c_int * 8)()
        assert N.lib().mvd_internal_fused_plan(ctx, 41, out) == N.MVD_ERR_UNSUPPORTED
    finally:
        api.mvd_destroy(ctx)
