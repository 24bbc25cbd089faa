"""Python binding of the plane-wise MV-RL library (same names as the C ABI).

The ``mvd_*`` functions marshal arguments for the C entry points of
``include/mvd.h``; PyTorch supplies device memory and the current HIP stream
only.  ``Deconvolver`` and ``deconvolve`` are conveniences over them.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, c_float, c_int, c_size_t, c_void_p

import numpy as np

from . import _native as N

__all__ = [
    "mvd_version", "mvd_create", "mvd_destroy", "mvd_set_psf", "mvd_get_back_taps",
    "mvd_psf_info", "mvd_workspace_bytes", "mvd_reslice", "mvd_deconvolve_planes",
    "mvd_get_timing", "mvd_last_error", "make_run", "Deconvolver", "deconvolve",
    "mvd_backward_workspace_bytes", "mvd_backward", "mvd_backward_grads", "mvd_batch_create", "mvd_batch_launch",
    "mvd_batch_tuning", "mvd_batch_destroy", "mvd_batch_run", "Batch",
    "mvd_stream_workspace_bytes", "mvd_deconvolve_stream", "mvd_deconvolve_planes_static",
    "mvd_batch_wait", "mvd_batch_info", "mvd_batch_form_times",
]


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def _dev_ptr(t):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA/HIP device tensor")
    if not t.is_contiguous():
        raise ValueError("device tensors must be contiguous")
    return c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# Thin wrappers of the C entry points
# ---------------------------------------------------------------------------
def mvd_version() -> int:
    return N.lib().mvd_version()


def mvd_last_error(ctx=None) -> str:
    return N.last_error(ctx)


def mvd_create(n_views: int, n_z: int, n_x: int, device: int = 0):
    ctx = c_void_p()
    N.check(N.lib().mvd_create(ctypes.byref(ctx), int(n_views), int(n_z), int(n_x), int(device)))
    return ctx


def mvd_destroy(ctx) -> None:
    N.lib().mvd_destroy(ctx)


def _host_f32(a, shape=None):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape is not None and arr.shape != shape:
        raise ValueError(f"expected shape {shape}, got {arr.shape}")
    return arr


def mvd_set_psf(ctx, view: int, taps, back_mode="flipped", back_taps=None) -> None:
    t = _host_f32(taps)
    if t.ndim != 2:
        raise ValueError("taps must be 2D [kz][kx]")
    mode = N.BACK[back_mode] if isinstance(back_mode, str) else int(back_mode)
    bt = None
    if back_taps is not None:
        bt = _host_f32(back_taps, t.shape)
    st = N.lib().mvd_set_psf(ctx, int(view), t.ctypes.data_as(POINTER(c_float)), t.shape[0], t.shape[1],
                             mode, bt.ctypes.data_as(POINTER(c_float)) if bt is not None else None)
    N.check(st, ctx)


def mvd_get_back_taps(ctx, view: int, kz: int, kx: int) -> np.ndarray:
    out = np.zeros((kz, kx), dtype=np.float32)
    N.check(N.lib().mvd_get_back_taps(ctx, int(view), out.ctypes.data_as(POINTER(c_float))), ctx)
    return out


def mvd_psf_info(ctx, view: int):
    """(PSF, back-projector) pass forms: 1 rank one, r ≥ 2 a sum of r rank-one
    terms, 0 K×K."""
    sp, sx = c_int(), c_int()
    N.check(N.lib().mvd_psf_info(ctx, int(view), ctypes.byref(sp), ctypes.byref(sx)), ctx)
    return sp.value, sx.value


def make_run(n_planes, n_iters, *, update="simultaneous", boundary="zero", init="mean",
             init_const=1.0, obs_dtype="f32", layout="stack_zyx", weights=None,
             checkpoints=None, workspace=None, workspace_bytes=0, force_2d=False, timing=False,
             graph=False, tune=False, normalize=False, weight_planes=None):
    """Build an ``mvd_run``; keeps host weight storage alive on the object.
    ``weight_planes``: per-view device pointers (or tensors) of per-pixel weights."""
    r = N.MvdRun()
    r.struct_size = ctypes.sizeof(N.MvdRun)
    r.flags = ((N.MVD_FLAG_FORCE_2D if force_2d else 0) | (N.MVD_FLAG_TIMING if timing else 0)
               | (N.MVD_FLAG_GRAPH if graph else 0) | (N.MVD_FLAG_TUNE if tune else 0)
               | (N.MVD_FLAG_NORMALIZE if normalize else 0))
    r.n_planes = int(n_planes)
    r.n_iters = int(n_iters)
    r.update = N.UPDATE[update]
    r.boundary = N.BOUNDARY[boundary]
    r.init = N.INIT[init]
    r.init_const = float(init_const)
    r.obs_dtype = {"u16": N.MVD_U16, "f32": N.MVD_F32}[obs_dtype]
    r.obs_layout = {"stack_zyx": N.MVD_STACK_ZYX, "planes_yzx": N.MVD_PLANES_YZX}[layout]
    if weights is not None:
        w = (c_float * len(weights))(*[float(x) for x in weights])
        r._weights_keepalive = w
        r.view_weights = ctypes.cast(w, POINTER(c_float))
    r.checkpoints = checkpoints
    r.workspace = workspace
    r.workspace_bytes = int(workspace_bytes)
    if weight_planes is not None:
        ptrs = [p.data_ptr() if hasattr(p, "data_ptr") else int(p) for p in weight_planes]
        arr = (ctypes.c_void_p * len(ptrs))(*ptrs)
        r._planes_keepalive = (arr, list(weight_planes))
        r.weight_planes = ctypes.cast(arr, ctypes.c_void_p)
    return r


def mvd_workspace_bytes(ctx, run) -> int:
    n = c_size_t()
    N.check(N.lib().mvd_workspace_bytes(ctx, ctypes.byref(run), ctypes.byref(n)), ctx)
    return n.value


def mvd_reslice(ctx, stack, n_planes: int, planes, stream=None) -> None:
    torch = _torch()
    dtype = {torch.uint16: N.MVD_U16, torch.float32: N.MVD_F32}[stack.dtype]
    N.check(N.lib().mvd_reslice(ctx, _dev_ptr(stack), dtype, int(n_planes), _dev_ptr(planes),
                                _stream_handle(stream)), ctx)


def mvd_get_timing(ctx, reset: bool = True) -> dict:
    """Summed launch times (ms) and counts of timed runs per launch kind."""
    t = N.MvdTiming()
    t.struct_size = ctypes.sizeof(N.MvdTiming)
    N.check(N.lib().mvd_get_timing(ctx, ctypes.byref(t), 1 if reset else 0), ctx)
    names = ("forward", "backward", "other", "adjoint", "correlation", "fused")
    return {n: (int(t.count[i]), float(t.ms[i])) for i, n in enumerate(names)}


def mvd_deconvolve_planes(ctx, obs, est, run, stream=None) -> None:
    ptrs = (c_void_p * len(obs))(*[_dev_ptr(o).value for o in obs])
    N.check(N.lib().mvd_deconvolve_planes(ctx, ptrs, _dev_ptr(est), ctypes.byref(run),
                                          _stream_handle(stream)), ctx)


def mvd_deconvolve_planes_static(ctx, obs, est, run, stream=None) -> None:
    """The allocation-free form: ``run`` carries no workspace (the library's
    static per-device scratch is used instead)."""
    ptrs = (c_void_p * len(obs))(*[_dev_ptr(o).value for o in obs])
    N.check(N.lib().mvd_deconvolve_planes_static(ctx, ptrs, _dev_ptr(est), ctypes.byref(run),
                                                 _stream_handle(stream)), ctx)


def _any_ptr(t):
    """Pointer of a contiguous device tensor or page-locked host tensor."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_contiguous():
        raise TypeError("expected a contiguous tensor")
    if not t.is_cuda and not t.is_pinned():
        raise ValueError("host tensors must be page-locked (pin_memory=True)")
    return c_void_p(t.data_ptr())


def mvd_stream_workspace_bytes(ctx, run, batch_planes: int, est_on_host: bool) -> int:
    n = c_size_t()
    N.check(N.lib().mvd_stream_workspace_bytes(ctx, ctypes.byref(run), int(batch_planes), int(bool(est_on_host)),
                                               ctypes.byref(n)), ctx)
    return n.value


def mvd_deconvolve_stream(ctx, obs, est, run, batch_planes: int, stream=None) -> None:
    """Streamed run: ``obs`` are camera-ordered stacks in page-locked host (or
    device) tensors, ``est`` a device or page-locked host tensor."""
    ptrs = (c_void_p * len(obs))(*[_any_ptr(o).value for o in obs])
    N.check(N.lib().mvd_deconvolve_stream(ctx, ptrs, _any_ptr(est), ctypes.byref(run), int(batch_planes),
                                          _stream_handle(stream)), ctx)


def mvd_deconvolve_files(ctx, obs_fds, est_fd, run, batch_planes: int, *, obs_offsets=None, est_offset=0,
                         host_slots=0, io_threads=0, sync=False, drop_cache=False, stream=None) -> dict:
    """Disk-to-disk run: camera-ordered stacks read from the open descriptors
    ``obs_fds`` (at ``obs_offsets``), ψ^T written as float32 planes to ``est_fd``
    at ``est_offset``; ``run.workspace`` is device memory of
    ``mvd_stream_workspace_bytes(ctx, run, batch_planes, True)`` bytes.  Returns
    the call's timings (s) and byte counts."""
    io = N.MvdFiles()
    io.struct_size = ctypes.sizeof(N.MvdFiles)
    io.flags = (N.MVD_FILES_SYNC if sync else 0) | (N.MVD_FILES_DROP_CACHE if drop_cache else 0)
    for v, fd in enumerate(obs_fds):
        io.obs_fd[v] = int(fd)
        io.obs_offset[v] = int(obs_offsets[v]) if obs_offsets is not None else 0
    io.est_fd = int(est_fd)
    io.est_offset = int(est_offset)
    io.host_slots = int(host_slots)
    io.io_threads = int(io_threads)
    N.check(N.lib().mvd_deconvolve_files(ctx, ctypes.byref(io), ctypes.byref(run), int(batch_planes),
                                         _stream_handle(stream)), ctx)
    return {"read_s": io.seconds[0], "write_s": io.seconds[1], "wait_s": io.seconds[2], "wall_s": io.seconds[3],
            "bytes_read": int(io.bytes[0]), "bytes_written": int(io.bytes[1])}


def mvd_backward_workspace_bytes(ctx, run) -> int:
    n = c_size_t()
    N.check(N.lib().mvd_backward_workspace_bytes(ctx, ctypes.byref(run), ctypes.byref(n)), ctx)
    return n.value


def _ptr_array(tensors):
    if tensors is None:
        return None
    return (c_void_p * len(tensors))(*[(_dev_ptr(t).value if t is not None else None) for t in tensors])


def mvd_backward(ctx, obs, grad_est, run, grad_psf=None, grad_back=None, grad_weights=None,
                 grad_init=None, stream=None) -> None:
    ptrs = (c_void_p * len(obs))(*[_dev_ptr(o).value for o in obs])
    gp = _ptr_array(grad_psf)
    gb = _ptr_array(grad_back)
    N.check(N.lib().mvd_backward(ctx, ptrs, _dev_ptr(grad_est), ctypes.byref(run),
                                 ctypes.cast(gp, POINTER(c_void_p)) if gp is not None else None,
                                 ctypes.cast(gb, POINTER(c_void_p)) if gb is not None else None,
                                 _dev_ptr(grad_weights) if grad_weights is not None else None,
                                 _dev_ptr(grad_init) if grad_init is not None else None,
                                 _stream_handle(stream)), ctx)


def mvd_backward_grads(ctx, obs, grad_est, run, grad_psf=None, grad_back=None, grad_weights=None,
                       grad_init=None, grad_weight_planes=None, stream=None) -> None:
    """mvd_backward with the per-pixel weight planes' gradients as well
    (`grad_weight_planes`: one float32 [Y][Z][X] device tensor per view)."""
    ptrs = (c_void_p * len(obs))(*[_dev_ptr(o).value for o in obs])
    keep = [_ptr_array(grad_psf), _ptr_array(grad_back), _ptr_array(grad_weight_planes)]
    g = N.MvdGrads()
    g.struct_size = ctypes.sizeof(N.MvdGrads)
    g.grad_psf = ctypes.cast(keep[0], POINTER(c_void_p)) if keep[0] is not None else None
    g.grad_back = ctypes.cast(keep[1], POINTER(c_void_p)) if keep[1] is not None else None
    g.grad_weights = _dev_ptr(grad_weights).value if grad_weights is not None else None
    g.grad_init = _dev_ptr(grad_init).value if grad_init is not None else None
    g.grad_weight_planes = ctypes.cast(keep[2], POINTER(c_void_p)) if keep[2] is not None else None
    N.check(N.lib().mvd_backward_grads(ctx, ptrs, _dev_ptr(grad_est), ctypes.byref(run), ctypes.byref(g),
                                       _stream_handle(stream)), ctx)


def _items(entries):
    """entries: [(ctx, obs tensors, est tensor, run)] → ctypes array + keep-alive list."""
    arr = (N.MvdItem * len(entries))()
    keep = []
    for i, (ctx, obs, est, run) in enumerate(entries):
        ptrs = (c_void_p * len(obs))(*[_dev_ptr(o).value for o in obs])
        keep.append(ptrs)
        arr[i].ctx = ctx
        arr[i].obs = ctypes.cast(ptrs, POINTER(c_void_p))
        arr[i].est = _dev_ptr(est)
        arr[i].run = ctypes.pointer(run)
        keep.append(run)
    return arr, keep


def mvd_batch_create(entries, tune=False, stream=None, graph=False):
    arr, keep = _items(entries)
    b = c_void_p()
    flags = (N.MVD_BATCH_TUNE if tune else 0) | (N.MVD_BATCH_GRAPH if graph else 0)
    N.check(N.lib().mvd_batch_create(ctypes.byref(b), arr, len(entries), flags, _stream_handle(stream)))
    return b


def mvd_batch_launch(b, stream=None) -> None:
    N.check(N.lib().mvd_batch_launch(b, _stream_handle(stream)))


def mvd_batch_wait(b, stream=None) -> None:
    N.check(N.lib().mvd_batch_wait(b, _stream_handle(stream)))


def mvd_batch_info(b):
    out = (c_int * 4)()
    N.check(N.lib().mvd_batch_info(b, out))
    return dict(persistent=bool(out[0]), items=out[1], work_groups=out[2], lds_bytes=out[3])


def mvd_batch_form_times(b):
    """(persistent ms, graph ms) measured by a tuned batch choosing its form, or (0, 0)."""
    out = (ctypes.c_double * 2)()
    N.check(N.lib().mvd_batch_form_times(b, out))
    return float(out[0]), float(out[1])


def mvd_batch_tuning(b, item: int):
    out = (c_int * 5)()
    N.check(N.lib().mvd_batch_tuning(b, int(item), out))
    return dict(fwd_occ=out[0], fwd_views=out[1], bwd_vin=out[2], zseg_scale=out[3], cols=out[4])


def mvd_batch_destroy(b) -> None:
    N.lib().mvd_batch_destroy(b)


def mvd_batch_run(entries, stream=None) -> None:
    arr, keep = _items(entries)
    N.check(N.lib().mvd_batch_run(arr, len(entries), _stream_handle(stream)))


class Batch:
    """Several deconvolutions in one launch: the persistent work-queue kernel,
    or a HIP graph with one branch per volume where items need it."""

    def __init__(self, entries, tune=False, stream=None, graph=False):
        self.entries = entries          # keeps tensors and runs alive
        self.handle = mvd_batch_create(entries, tune, stream, graph)

    def launch(self, stream=None):
        mvd_batch_launch(self.handle, stream)

    def wait(self, stream=None):
        mvd_batch_wait(self.handle, stream)

    def info(self):
        return mvd_batch_info(self.handle)

    def tuning(self, item):
        return mvd_batch_tuning(self.handle, item)

    def form_times(self):
        return mvd_batch_form_times(self.handle)

    def close(self):
        if self.handle is not None:
            mvd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Convenience layer
# ---------------------------------------------------------------------------
class Deconvolver:
    """A context for V views of Z×X planes with its PSFs set."""

    def __init__(self, n_views: int, n_z: int, n_x: int, device: int = 0):
        self.n_views, self.n_z, self.n_x, self.device = n_views, n_z, n_x, device
        self.ctx = mvd_create(n_views, n_z, n_x, device)
        self.psf_shapes = [None] * n_views

    def close(self):
        if self.ctx is not None:
            mvd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check_tensors(self, obs, layout, *, iters, est=None, checkpoints=None, weight_planes=None):
        """Check the tensors of a run against this context before any pointer
        reaches the library: one observation per view, all uint16 or all
        float32 of the layout's shape (camera stack [Z][Y][X] or planes
        [Y][Z][X]) on one device; est float32 [Y][Z][X]; checkpoints float32
        with T·Y·Z·X elements; weight planes float32 [Y][Z][X].  Returns
        (Y, obs dtype name); raises ValueError / TypeError."""
        torch = _torch()
        if len(obs) != self.n_views:
            raise ValueError(f"one observation tensor per view ({self.n_views}), got {len(obs)}")
        if layout not in ("stack_zyx", "planes_yzx"):
            raise ValueError(f"unknown layout {layout!r}")
        o0 = obs[0]
        if not isinstance(o0, torch.Tensor) or o0.dim() != 3:
            raise ValueError("observations must be 3D tensors")
        if o0.dtype not in (torch.uint16, torch.float32):
            raise TypeError(f"observations must be uint16 or float32, got {o0.dtype}")
        n_planes = o0.shape[1] if layout == "stack_zyx" else o0.shape[0]
        want = (self.n_z, n_planes, self.n_x) if layout == "stack_zyx" else (n_planes, self.n_z, self.n_x)
        for v, o in enumerate(obs):
            if not isinstance(o, torch.Tensor) or o.dtype != o0.dtype:
                raise TypeError(f"view {v}: every view must have the dtype of view 0 ({o0.dtype})")
            if tuple(o.shape) != want:
                raise ValueError(f"view {v}: shape {tuple(o.shape)} != {want} for layout {layout}")
            if o.device != o0.device:
                raise ValueError(f"view {v}: all views must be on one device")
        plane_shape = (n_planes, self.n_z, self.n_x)

        def f32_of(t, name, shape=None, numel=None):
            if not isinstance(t, torch.Tensor) or t.dtype != torch.float32:
                raise TypeError(f"{name} must be a float32 tensor")
            if shape is not None and tuple(t.shape) != shape:
                raise ValueError(f"{name}: shape {tuple(t.shape)} != {shape}")
            if numel is not None and t.numel() != numel:
                raise ValueError(f"{name}: {t.numel()} elements, need {numel}")
            if t.device != o0.device:
                raise ValueError(f"{name} must be on the observations' device")

        if est is not None:
            f32_of(est, "est", shape=plane_shape)
        if checkpoints is not None:
            f32_of(checkpoints, "checkpoints", numel=int(iters) * n_planes * self.n_z * self.n_x)
        if weight_planes is not None:
            if len(weight_planes) != self.n_views:
                raise ValueError("one weight plane set per view")
            for v, w in enumerate(weight_planes):
                f32_of(w, f"weight_planes[{v}]", shape=plane_shape)
        return n_planes, ("u16" if o0.dtype == torch.uint16 else "f32")

    def set_psf(self, view, taps, back="flipped", back_taps=None):
        mvd_set_psf(self.ctx, view, taps, back, back_taps)
        self.psf_shapes[view] = np.asarray(taps).shape

    def back_taps(self, view):
        kz, kx = self.psf_shapes[view]
        return mvd_get_back_taps(self.ctx, view, kz, kx)

    def run(self, obs, *, iters, est=None, update="simultaneous", boundary="zero", init="mean",
            init_const=1.0, weights=None, layout=None, checkpoints=None, force_2d=False,
            stream=None, normalize=False, weight_planes=None):
        """Deconvolve device observations; returns the estimate ``[Y][Z][X]`` (float32)."""
        torch = _torch()
        if layout is None:
            layout = "stack_zyx"
        n_planes, obs_dtype = self.check_tensors(obs, layout, iters=iters, est=est, checkpoints=checkpoints,
                                                 weight_planes=weight_planes)
        o0 = obs[0]
        if est is None:
            est = torch.empty((n_planes, self.n_z, self.n_x), dtype=torch.float32, device=o0.device)
        run = make_run(n_planes, iters, update=update, boundary=boundary, init=init,
                       init_const=init_const, obs_dtype=obs_dtype, layout=layout, weights=weights,
                       force_2d=force_2d, normalize=normalize, weight_planes=weight_planes,
                       checkpoints=checkpoints.data_ptr() if checkpoints is not None else None)
        nbytes = mvd_workspace_bytes(self.ctx, run)
        ws = None
        if nbytes:
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=o0.device)
            base = ws.data_ptr()
            run.workspace = (base + 255) // 256 * 256
            run.workspace_bytes = nbytes
        mvd_deconvolve_planes(self.ctx, obs, est, run, stream)
        if ws is not None:
            s = stream if stream is not None else torch.cuda.current_stream()
            ws.record_stream(s)
        return est


def deconvolve(obs, psfs, *, iters=10, update="simultaneous", boundary="zero", back="flipped",
               back_taps=None, weights=None, init="mean", init_const=1.0, est=None,
               layout="stack_zyx", force_2d=False, stream=None, normalize=False, weight_planes=None):
    """One-shot plane-wise MV-RL on device tensors; returns ψ^T ``[Y][Z][X]``."""
    o0 = obs[0]
    if layout == "stack_zyx":
        nz, nx = o0.shape[0], o0.shape[2]
    else:
        nz, nx = o0.shape[1], o0.shape[2]
    dev = o0.device.index if o0.device.index is not None else 0
    d = Deconvolver(len(obs), nz, nx, dev)
    try:
        for v, p in enumerate(psfs):
            d.set_psf(v, p, back, None if back_taps is None else back_taps[v])
        out = d.run(obs, iters=iters, est=est, update=update, boundary=boundary, init=init,
                    init_const=init_const, weights=weights, layout=layout, force_2d=force_2d,
                    stream=stream, normalize=normalize, weight_planes=weight_planes)
        # the context's device taps must outlive the enqueued work
        (stream if stream is not None else _torch().cuda.current_stream()).synchronize()
        return out
    finally:
        d.close()
