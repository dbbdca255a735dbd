"""Continuous Fourier series of rectilinear polygons on MI355X (gfx950).

Thin Python binding over the C ABI of ``include/fcfs.h``: it only marshals
arguments.  Every step of the transform runs in the HIP kernels of
``libfcfs.so``; PyTorch supplies device memory and the current stream.
Importing works without a GPU; every entry point that touches the device
raises if the library or the device is missing.
"""
from __future__ import annotations

import ctypes
import functools

import numpy as np

from ._lib import (PRECISIONS, FcfsClip, FcfsError, FcfsGClip, FcfsHaarClip, check,  # noqa: F401
                   load)

__all__ = [
    "Handle", "FcfsError", "loops_to_corners", "forward", "workspace_size", "debug_phases",
    "tile_variants", "PRECISIONS", "haar", "forward_general", "adjoint_general",
]


def _prec(p) -> int:
    if isinstance(p, int):
        return p
    try:
        return PRECISIONS[p]
    except KeyError:
        raise ValueError(f"unknown precision {p!r}; one of {sorted(PRECISIONS)}") from None


def loops_to_corners(xy, off):
    """Polygon loops -> (x, y, s, hedge, vedge) numpy arrays (host; a1 of the path).

    ``xy``: (n, 2) int32 lattice coordinates, ``off``: (n_loops+1,) int64.
    """
    lib = load()
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.int32).reshape(-1, 2))
    off = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    n = xy.shape[0]
    x = np.empty(n, np.int32)
    y = np.empty(n, np.int32)
    s = np.empty(n, np.int8)
    he = np.empty(n, np.int64)
    ve = np.empty(n, np.int64)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    check(lib.fcfs_loops_to_corners(p(xy), p(off), off.size - 1, p(x), p(y), p(s), p(he), p(ve)))
    return x, y, s, he, ve


def tile_variants():
    """[(wk, wl)] frequencies per wave of every contraction tile variant."""
    lib = load()
    n = lib.fcfs_tile_variants(None, None, 0)
    wk = (ctypes.c_int32 * n)()
    wl = (ctypes.c_int32 * n)()
    lib.fcfs_tile_variants(wk, wl, n)
    return list(zip(wk, wl))


def _clip(x, y, s, V, T, K, L, F=None, area=None) -> FcfsClip:
    c = FcfsClip()
    c.x = x.data_ptr() if x is not None else None
    c.y = y.data_ptr() if y is not None else None
    c.s = s.data_ptr() if s is not None else None
    c.V, c.T, c.K, c.L = int(V), int(T), int(K), int(L)
    c.F = F.data_ptr() if F is not None else None
    c.area = area.data_ptr() if area is not None else None
    return c


@functools.lru_cache(maxsize=256)
def workspace_size(V: int, T: int, K: int, L: int, precision="bf16", adjoint: bool = False,
                   tile: int | None = None) -> int:
    lib = load()
    c = _clip(None, None, None, V, T, K, L)
    n = ctypes.c_size_t(0)
    if tile is None:
        check(lib.fcfs_workspace_size(ctypes.byref(c), _prec(precision), int(adjoint),
                                      ctypes.byref(n)))
    else:
        check(lib.fcfs_workspace_size_tile(ctypes.byref(c), _prec(precision), int(tile),
                                           ctypes.byref(n)))
    return int(n.value)


def forward_noalloc(x, y, s, T: int, K: int, L: int | None = None, precision="bf16",
                    handle=None, out=None, area_out=None):
    """``forward`` through ``fcfs_forward_noalloc``: the library's own scratch on
    the device replaces the workspace (clips up to its size).  Returns
    ``(F, area)``; ``out`` / ``area_out`` may supply the output tensors."""
    import torch

    L = K if L is None else L
    h = handle or default_handle()
    h.sync_stream()
    x, y, s = _corners_on(h.device, x, y, s)
    V = x.numel()
    F = out if out is not None else torch.empty((2 * K + 1, 2 * L + 1), dtype=torch.complex64,
                                                 device=h.device)
    a = area_out if area_out is not None else torch.empty(1, dtype=torch.int64, device=h.device)
    c = _clip(x, y, s, V, T, K, L, F, a)
    check(h.lib.fcfs_forward_noalloc(h.ptr, ctypes.byref(c), _prec(precision)), h.ptr)
    return F, a


def plan_info(V: int, T: int, K: int, L: int, precision="bf16") -> dict:
    """The automatic plan of ``forward`` for these sizes (``fcfs_forward_plan_info``):
    vertex splits, corners per split, frequency tiles, direct form, and the form
    taken ("contraction", "direct" or, for precision "auto", "lattice")."""
    lib = load()
    c = _clip(None, None, None, V, T, K, L)
    ns, ti, di = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    ch = ctypes.c_int64(0)
    check(lib.fcfs_forward_plan_info(ctypes.byref(c), _prec(precision), ctypes.byref(ns),
                                     ctypes.byref(ch), ctypes.byref(ti), ctypes.byref(di)))
    return {"nsplit": ns.value, "chunk": ch.value, "tiles": ti.value, "direct": di.value == 1,
            "form": ("contraction", "direct", "lattice")[di.value]}


class Handle:
    """Owns an ``fcfs_handle`` (twiddle tables) on one device.

    Each call enqueues on torch's current stream; on a change of stream the
    library orders the new stream after the old one, so the cached workspace
    is never used by two streams at once.  Calls through one handle must not
    overlap in time (autograd's backward thread uses it while the caller
    waits)."""

    def __init__(self, device=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("paper_1010_5562_amd needs a ROCm GPU; none is visible")
        self.lib = load()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.device = dev
        self._h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(dev).cuda_stream
        check(self.lib.fcfs_create(ctypes.byref(self._h), dev.index, ctypes.c_void_p(stream)))
        self._stream = stream
        self._ws = None

    def close(self):
        if self._h:
            self.lib.fcfs_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ptr(self):
        return self._h

    def sync_stream(self):
        import torch

        stream = torch.cuda.current_stream(self.device).cuda_stream
        if stream != self._stream:
            check(self.lib.fcfs_set_stream(self._h, ctypes.c_void_p(stream)), self._h)
            self._stream = stream

    def set_tile(self, variant: int = -1):
        check(self.lib.fcfs_set_tile(self._h, int(variant)), self._h)

    PROFILE_KINDS = ("prepass", "axis", "contract", "epilogue", "adjoint", "batch", "fft",
                     "haar", "loss", "direct", "step", "adjoint_gemm")

    def profile_begin(self, kinds=None):
        """Starts event timing of the named kinds (all kinds when None)."""
        mask = 0
        for k in kinds or ():
            mask |= 1 << self.PROFILE_KINDS.index(k)
        check(self.lib.fcfs_profile_begin(self._h, mask), self._h)

    def profile_end(self):
        """{kind: (total_ms, launches)} since profile_begin (waits for the events)."""
        n = len(self.PROFILE_KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        check(self.lib.fcfs_profile_end(self._h, ms, cnt, n), self._h)
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.PROFILE_KINDS)}

    def workspace(self, nbytes: int):
        """A cached device workspace of at least ``nbytes`` (256-byte aligned)."""
        import torch

        if self._ws is None or self._ws.numel() < nbytes:
            if self._ws is not None:
                # the old buffer returns to the pool of the stream it was
                # allocated on; work already enqueued on the current one may
                # still read it
                self._ws.record_stream(torch.cuda.current_stream(self.device))
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self._ws


_default = {}


def default_handle(device=None) -> Handle:
    import torch

    idx = torch.cuda.current_device() if device is None else torch.device(device).index
    h = _default.get(idx)
    if h is None:
        h = _default[idx] = Handle(idx)
    return h


def _on(dev, a, dtype):
    import torch

    if isinstance(a, torch.Tensor) and a.dtype == dtype and a.device == dev and a.is_contiguous():
        return a
    return torch.as_tensor(a, dtype=dtype).to(dev).contiguous()


def _corners_on(dev, x, y, s):
    import torch

    x = _on(dev, x, torch.int32)
    y = _on(dev, y, torch.int32)
    s = _on(dev, s, torch.int8)
    if not (x.numel() == y.numel() == s.numel()):
        raise ValueError("x, y, s differ in length")
    return x, y, s


def forward(x, y, s, T: int, K: int, L: int | None = None, precision="bf16", handle=None,
            out=None, area_out=None, tile: int | None = None, band=None, radius=None):
    """CFS coefficients F[k, l], |k| <= K, |l| <= L, of a signed corner list.

    Returns ``(F, area)``: F a (2K+1, 2L+1) complex64 tensor indexed
    [k + K, l + L], area a 1-element int64 tensor (exact sum s x y).
    ``band=(kmax, lmax)`` and/or ``radius`` restrict the computation to
    |k| <= kmax, |l| <= lmax and k^2 + l^2 <= radius^2 (``fcfs_forward_band``);
    the other entries of F are zero.
    """
    import torch

    L = K if L is None else L
    h = handle or default_handle()
    h.sync_stream()
    x, y, s = _corners_on(h.device, x, y, s)
    V = x.numel()
    F = out if out is not None else torch.empty((2 * K + 1, 2 * L + 1), dtype=torch.complex64,
                                                device=h.device)
    if F.dtype != torch.complex64 or F.numel() != (2 * K + 1) * (2 * L + 1) or not F.is_contiguous():
        raise ValueError("out must be a contiguous complex64 tensor of (2K+1)(2L+1) entries")
    area = area_out if area_out is not None else torch.empty(1, dtype=torch.int64, device=h.device)
    if tile is not None:
        h.set_tile(tile)
    try:
        c = _clip(x, y, s, V, T, K, L, F, area)
        if band is None and radius is None:
            nbytes = workspace_size(V, T, K, L, precision, tile=tile)
            ws = h.workspace(nbytes)
            check(h.lib.fcfs_forward(h.ptr, ctypes.byref(c), _prec(precision),
                                     ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel())),
                  h.ptr)
        else:
            kmax, lmax = (K, L) if band is None else (int(band[0]), int(band[1]))
            rad = -1.0 if radius is None else float(radius)
            ws = h.workspace(_band_workspace_size(V, T, K, L, kmax, lmax, rad, _prec(precision)))
            check(h.lib.fcfs_forward_band(h.ptr, ctypes.byref(c), kmax, lmax, rad,
                                          _prec(precision), ctypes.c_void_p(ws.data_ptr()),
                                          ctypes.c_size_t(ws.numel())), h.ptr)
    finally:
        if tile is not None:
            h.set_tile(-1)
    return F, area


def forward_fft(x, y, s, T: int, K: int, L: int | None = None, handle=None, out=None,
                area_out=None):
    """The same coefficients as ``forward`` from the lattice (FFT) form in FP64
    (``fcfs_forward_fft``).  Returns ``(F, area)``."""
    import torch

    L = K if L is None else L
    h = handle or default_handle()
    h.sync_stream()
    x, y, s = _corners_on(h.device, x, y, s)
    V = x.numel()
    F = out if out is not None else torch.empty((2 * K + 1, 2 * L + 1), dtype=torch.complex64,
                                                device=h.device)
    if F.dtype != torch.complex64 or F.numel() != (2 * K + 1) * (2 * L + 1) or not F.is_contiguous():
        raise ValueError("out must be a contiguous complex64 tensor of (2K+1)(2L+1) entries")
    area = area_out if area_out is not None else torch.empty(1, dtype=torch.int64, device=h.device)
    c = _clip(x, y, s, V, T, K, L, F, area)
    nb = ctypes.c_size_t(0)
    check(h.lib.fcfs_fft_workspace_size(ctypes.byref(c), ctypes.byref(nb)))
    ws = h.workspace(nb.value)
    check(h.lib.fcfs_forward_fft(h.ptr, ctypes.byref(c), ctypes.c_void_p(ws.data_ptr()),
                                 ctypes.c_size_t(ws.numel())), h.ptr)
    return F, area


def forward_general(x, y, s, Nx: int, Ny: int, K: int, L: int | None = None, frac_bits: int = 0,
                    precision="bf16", handle=None, out=None, area_out=None, band=None,
                    radius=None):
    """Coefficients of a general tile (``fcfs_forward_general``): periods Nx,
    Ny (any integers), corners on the grid of step 2^-frac_bits given as
    integers (true coordinate times 2^frac_bits).  Returns ``(F, area)`` as
    ``forward``; area is sum s x y in grid units (the area times
    4^frac_bits).  ``band`` and ``radius`` as for ``forward``
    (``fcfs_forward_general_band``)."""
    import torch

    L = K if L is None else L
    h = handle or default_handle()
    h.sync_stream()
    x, y, s = _corners_on(h.device, x, y, s)
    F = out if out is not None else torch.empty((2 * K + 1, 2 * L + 1), dtype=torch.complex64,
                                                device=h.device)
    if F.dtype != torch.complex64 or F.numel() != (2 * K + 1) * (2 * L + 1) or not F.is_contiguous():
        raise ValueError("out must be a contiguous complex64 tensor of (2K+1)(2L+1) entries")
    area = area_out if area_out is not None else torch.empty(1, dtype=torch.int64, device=h.device)
    c = FcfsGClip(x.data_ptr(), y.data_ptr(), s.data_ptr(), x.numel(), int(Nx), int(Ny),
                  int(frac_bits), int(K), int(L), F.data_ptr(), area.data_ptr())
    nb = ctypes.c_size_t(0)
    if band is None and radius is None:
        check(h.lib.fcfs_general_workspace_size(ctypes.byref(c), _prec(precision),
                                                ctypes.byref(nb)))
        ws = h.workspace(nb.value)
        check(h.lib.fcfs_forward_general(h.ptr, ctypes.byref(c), _prec(precision),
                                         ctypes.c_void_p(ws.data_ptr()),
                                         ctypes.c_size_t(ws.numel())), h.ptr)
    else:
        kmax, lmax = (K, L) if band is None else (int(band[0]), int(band[1]))
        rad = -1.0 if radius is None else float(radius)
        check(h.lib.fcfs_general_band_workspace_size(ctypes.byref(c), kmax, lmax, rad,
                                                     _prec(precision), ctypes.byref(nb)))
        ws = h.workspace(nb.value)
        check(h.lib.fcfs_forward_general_band(h.ptr, ctypes.byref(c), kmax, lmax, rad,
                                              _prec(precision), ctypes.c_void_p(ws.data_ptr()),
                                              ctypes.c_size_t(ws.numel())), h.ptr)
    return F, area


def adjoint_general(x, y, s, Nx: int, Ny: int, K: int, L: int, grad_F, frac_bits: int = 0,
                    precision="bf16", band=None, radius=None, handle=None):
    """dLoss/dx_v, dLoss/dy_v (lattice units) of a general tile
    (``fcfs_adjoint_general``); x, y in grid units as for
    ``forward_general``, band and radius as for ``adjoint``."""
    import torch

    h = handle or default_handle()
    h.sync_stream()
    x, y, s = _corners_on(h.device, x, y, s)
    V = x.numel()
    G = torch.as_tensor(grad_F).to(h.device, torch.complex64).contiguous()
    if G.numel() != (2 * K + 1) * (2 * L + 1):
        raise ValueError("grad_F must have (2K+1)(2L+1) entries")
    gx = torch.empty(V, dtype=torch.float32, device=h.device)
    gy = torch.empty(V, dtype=torch.float32, device=h.device)
    kmax, lmax = (K, L) if band is None else (int(band[0]), int(band[1]))
    c = FcfsGClip(x.data_ptr(), y.data_ptr(), s.data_ptr(), V, int(Nx), int(Ny), int(frac_bits),
                  int(K), int(L), None, None)
    nb = ctypes.c_size_t(0)
    check(h.lib.fcfs_general_adjoint_workspace_size(ctypes.byref(c), _prec(precision),
                                                    ctypes.byref(nb)))
    ws = h.workspace(nb.value)
    check(h.lib.fcfs_adjoint_general(h.ptr, ctypes.byref(c), ctypes.c_void_p(G.data_ptr()), kmax,
                                     lmax, -1.0 if radius is None else float(radius),
                                     ctypes.c_void_p(gx.data_ptr()), ctypes.c_void_p(gy.data_ptr()),
                                     _prec(precision), ctypes.c_void_p(ws.data_ptr()),
                                     ctypes.c_size_t(ws.numel())), h.ptr)
    return gx, gy


def haar(x, y, s, poly_off, Nx: int, Ny: int, J: int, handle=None, out_U=None, out_W=None,
         coefficients: bool = True, stats: bool = False):
    """Pruned continuous Haar transform of one tile (``fcfs_haar``).

    x, y, s: corners in loop order (``loops_to_corners``); poly_off: the
    (M + 1,) int64 polygon offsets into them.  Returns ``(U, W, st)``: U the
    2^J x 2^J int64 pyramid of integer sums, W the float64 coefficients (None
    unless ``coefficients``), st a 2-element int64 tensor (cells visited,
    cell-corner pairs) or None."""
    import torch

    h = handle or default_handle()
    h.sync_stream()
    x, y, s = _corners_on(h.device, x, y, s)
    off = torch.as_tensor(poly_off, dtype=torch.int64).to(h.device).contiguous()
    side = 1 << int(J)
    U = out_U if out_U is not None else torch.empty((side, side), dtype=torch.int64,
                                                    device=h.device)
    if U.dtype != torch.int64 or U.numel() != side * side or not U.is_contiguous():
        raise ValueError("out_U must be a contiguous int64 tensor of 4^J entries")
    W = None
    if coefficients:
        W = out_W if out_W is not None else torch.empty((side, side), dtype=torch.float64,
                                                        device=h.device)
        if W.dtype != torch.float64 or W.numel() != side * side or not W.is_contiguous():
            raise ValueError("out_W must be a contiguous float64 tensor of 4^J entries")
    st = torch.empty(2, dtype=torch.int64, device=h.device) if stats else None
    c = FcfsHaarClip(x.data_ptr(), y.data_ptr(), s.data_ptr(), off.data_ptr(), x.numel(),
                     max(0, off.numel() - 1), int(Nx), int(Ny), int(J), U.data_ptr(),
                     W.data_ptr() if W is not None else None,
                     st.data_ptr() if st is not None else None)
    nb = ctypes.c_size_t(0)
    check(h.lib.fcfs_haar_workspace_size(ctypes.byref(c), ctypes.byref(nb)))
    ws = h.workspace(nb.value)
    check(h.lib.fcfs_haar(h.ptr, ctypes.byref(c), ctypes.c_void_p(ws.data_ptr()),
                          ctypes.c_size_t(ws.numel())), h.ptr)
    return U, W, st


def debug_phases(x, y, s, T: int, k0: int, nk: int, axis: int = 0, handle=None):
    """Exact integer phases (k0+i) * x_v mod T (axis 0) or with y_v (axis 1),
    as the contraction computes them; an (nk, V) int32 tensor."""
    import torch

    h = handle or default_handle()
    h.sync_stream()
    x, y, s = _corners_on(h.device, x, y, s)
    V = x.numel()
    p = torch.empty((nk, V), dtype=torch.int32, device=h.device)
    c = _clip(x, y, s, V, T, 0, 0)
    nb = ctypes.c_size_t(0)
    check(h.lib.fcfs_debug_phases_workspace_size(V, int(T), ctypes.byref(nb)))
    ws = h.workspace(nb.value)
    check(h.lib.fcfs_debug_phases(h.ptr, ctypes.byref(c), int(axis), int(k0), int(nk),
                                  ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                  ctypes.c_size_t(ws.numel())), h.ptr)
    return p


def adjoint(x, y, s, T: int, K: int, L: int, grad_F, precision="bf16", band=None, handle=None,
            radius=None):
    """dLoss/dx_v and dLoss/dy_v for a cotangent grad_F = dLoss/dRe F + j dLoss/dIm F
    ((2K+1, 2L+1) complex64).  band = (kmax, lmax) and radius restrict the work
    (and the entries of grad_F used) to |k| <= kmax, |l| <= lmax,
    k^2 + l^2 <= radius^2: the adjoint of ``forward`` with the same band and
    radius.  Returns (gx, gy) float32 tensors of length V."""
    import torch

    h = handle or default_handle()
    h.sync_stream()
    x, y, s = _corners_on(h.device, x, y, s)
    V = x.numel()
    G = _on(h.device, grad_F, torch.complex64)
    if G.numel() != (2 * K + 1) * (2 * L + 1):
        raise ValueError("grad_F must have (2K+1)(2L+1) entries")
    gx = torch.empty(V, dtype=torch.float32, device=h.device)
    gy = torch.empty(V, dtype=torch.float32, device=h.device)
    kmax, lmax = (K, L) if band is None else (int(band[0]), int(band[1]))
    nbytes = workspace_size(V, T, K, L, precision, adjoint=True)
    ws = h.workspace(nbytes)
    c = _clip(x, y, s, V, T, K, L)
    rad = -1.0 if radius is None else float(radius)
    check(h.lib.fcfs_adjoint_band(h.ptr, ctypes.byref(c), ctypes.c_void_p(G.data_ptr()), kmax, lmax,
                                  rad, ctypes.c_void_p(gx.data_ptr()), ctypes.c_void_p(gy.data_ptr()),
                                  _prec(precision), ctypes.c_void_p(ws.data_ptr()),
                                  ctypes.c_size_t(ws.numel())), h.ptr)
    return gx, gy


def edge_grad(gx, gy, hedge, vedge, n_edges: int, handle=None):
    """Edge-offset gradient: the sum over the two corners of each edge of gx
    (vertical edges) or gy (horizontal edges)."""
    import torch

    h = handle or default_handle()
    h.sync_stream()
    dev = h.device
    hedge = _on(dev, hedge, torch.int64)
    vedge = _on(dev, vedge, torch.int64)
    g = torch.empty(int(n_edges), dtype=torch.float32, device=dev)
    check(h.lib.fcfs_edge_grad(h.ptr, ctypes.c_void_p(gx.data_ptr()), ctypes.c_void_p(gy.data_ptr()),
                               ctypes.c_void_p(hedge.data_ptr()), ctypes.c_void_p(vedge.data_ptr()),
                               gx.numel(), int(n_edges), ctypes.c_void_p(g.data_ptr())), h.ptr)
    return g


class Geometry:
    """Device-resident polygon geometry for edge-moving optimisation: base
    corner coordinates, corner signs and the corner -> edge maps.

    Square tile: period T (a power of two), integer corners, integer edge
    offsets.  General tile (``Ny`` given, T not a power of two, or
    ``frac_bits`` > 0): periods T x Ny and corners on the grid of step
    2^-frac_bits (``xy`` holds the true coordinates); edge offsets are then
    multiples of 2^-frac_bits.

    ``check_offsets``: offsets off that grid raise FcfsError (a comparison
    that waits for the device on every call); with False they are rounded to
    the nearest grid point (ties to even) on the device and nothing waits,
    for loops whose offsets lie on the grid by construction."""

    def __init__(self, xy, off, T: int, K: int, L: int | None = None, handle=None,
                 Ny: int | None = None, frac_bits: int = 0, check_offsets: bool = True):
        import torch

        self.check_offsets = bool(check_offsets)
        self.handle = handle or default_handle()
        dev = self.handle.device
        self.frac_bits = int(frac_bits)
        self.T, self.K, self.L = int(T), int(K), int(K if L is None else L)
        self.Ny = int(T if Ny is None else Ny)
        self.general = (Ny is not None or self.frac_bits > 0 or self.T & (self.T - 1) != 0)
        xyg = np.asarray(xy, dtype=np.float64) * (1 << self.frac_bits)
        if not np.array_equal(xyg, np.round(xyg)):
            raise ValueError("corners must lie on the grid of step 2^-frac_bits")
        x, y, s, he, ve = loops_to_corners(np.round(xyg).astype(np.int32), off)
        self.n_edges = int(x.size)
        self.base_x = torch.as_tensor(x).to(dev)
        self.base_y = torch.as_tensor(y).to(dev)
        self.s = torch.as_tensor(s).to(dev)
        self.hedge = torch.as_tensor(he).to(dev)
        self.vedge = torch.as_tensor(ve).to(dev)

    def corners(self, offsets):
        """Corner coordinates (grid units) for edge offsets (one per edge, on
        the grid of step 2^-frac_bits)."""
        import torch

        h = self.handle
        h.sync_stream()
        off = offsets.detach().to(h.device, torch.float32).contiguous()
        if off.numel() != self.n_edges:
            raise ValueError("one offset per edge")
        sc = float(1 << self.frac_bits)
        if self.check_offsets and not torch.equal(off * sc, torch.round(off * sc)):
            raise FcfsError(-1, "edge offsets must be multiples of 2^-frac_bits")
        V = self.base_x.numel()
        x = torch.empty_like(self.base_x)
        y = torch.empty_like(self.base_y)
        args = (ctypes.c_void_p(self.base_x.data_ptr()), ctypes.c_void_p(self.base_y.data_ptr()),
                ctypes.c_void_p(self.hedge.data_ptr()), ctypes.c_void_p(self.vedge.data_ptr()),
                ctypes.c_void_p(off.data_ptr()), V)
        if self.general:
            check(h.lib.fcfs_apply_edge_offsets_grid(h.ptr, *args, self.frac_bits,
                                                     ctypes.c_void_p(x.data_ptr()),
                                                     ctypes.c_void_p(y.data_ptr())), h.ptr)
        else:
            check(h.lib.fcfs_apply_edge_offsets(h.ptr, *args, ctypes.c_void_p(x.data_ptr()),
                                                ctypes.c_void_p(y.data_ptr())), h.ptr)
        return x, y


def pupil_step(geom, offsets, G, radius=None, band=None, H=None, precision="bf16", F_out=None):
    """One optimisation step behind a pupil in a single library call
    (``fcfs_pupil_step``): corners moved by ``offsets`` (one per edge, rounded
    to integers), low-pass forward over ``band`` / ``radius``, loss
    sum |H F - G|^2 (H the disc indicator when None), adjoint and edge
    reduction.  The same launches as ``FCFSFunction`` + ``PupilLoss`` +
    ``backward()``, without the autograd engine.  Square tiles only.
    Returns ``(loss, g_edge)``: a 0-d float64 tensor and the float32 edge
    gradient; the spectrum goes to ``F_out`` when given."""
    import torch

    if geom.general:
        raise NotImplementedError("pupil_step takes square power-of-two tiles")
    h = geom.handle
    h.sync_stream()
    dev = h.device
    V, T, K, L = geom.n_edges, geom.T, geom.K, geom.L
    off = _on(dev, offsets.detach() if isinstance(offsets, torch.Tensor) else offsets,
              torch.float32)
    G = _on(dev, G, torch.complex64)
    Hc = None if H is None else _on(dev, H, torch.float32)
    if off.numel() != V or G.numel() != (2 * K + 1) * (2 * L + 1):
        raise ValueError("one offset per edge and a (2K+1, 2L+1) target")
    if F_out is not None and (F_out.dtype != torch.complex64 or F_out.numel() != G.numel()
                              or not F_out.is_contiguous()):
        raise ValueError("F_out must be a contiguous complex64 tensor like G")
    kmax, lmax = (K, L) if band is None else (int(band[0]), int(band[1]))
    rad = -1.0 if radius is None else float(radius)
    loss = torch.empty((), dtype=torch.float64, device=dev)
    g = torch.empty(V, dtype=torch.float32, device=dev)
    ws = h.workspace(_step_workspace_size(V, T, K, L, kmax, lmax, rad, _prec(precision)))
    vp = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())  # noqa: E731
    check(h.lib.fcfs_pupil_step(h.ptr, vp(geom.base_x), vp(geom.base_y), vp(geom.s),
                                vp(geom.hedge), vp(geom.vedge), vp(off), V, T, K, L, kmax, lmax,
                                rad, vp(G), vp(Hc), _prec(precision), vp(loss), vp(g), vp(F_out),
                                vp(ws), ctypes.c_size_t(ws.numel())), h.ptr)
    return loss, g


class PupilStep:
    """``pupil_step`` captured once into a graph (``fcfs_pupil_step_plan``)
    and replayed by ``run(offsets)``: the offsets are copied into the plan's
    own buffer, then the graph runs on the current stream.  ``loss``,
    ``g_edge`` and ``F`` are the plan's output tensors, overwritten by every
    run; G (and H) are copied at construction, and ``G.copy_(...)`` between
    runs changes the target.  The plan holds its own workspace."""

    def __init__(self, geom, G, radius=None, band=None, H=None, precision="bf16"):
        import torch

        if geom.general:
            raise NotImplementedError("PupilStep takes square power-of-two tiles")
        self.geom = geom
        h = self.handle = geom.handle
        h.sync_stream()
        dev = h.device
        V, T, K, L = geom.n_edges, geom.T, geom.K, geom.L
        self.offsets = torch.zeros(V, dtype=torch.float32, device=dev)
        self.G = _on(dev, G, torch.complex64).clone()
        if self.G.numel() != (2 * K + 1) * (2 * L + 1):
            raise ValueError("G must have (2K+1)(2L+1) entries")
        self.H = None if H is None else _on(dev, H, torch.float32).clone()
        self.loss = torch.empty((), dtype=torch.float64, device=dev)
        self.g_edge = torch.empty(V, dtype=torch.float32, device=dev)
        self.F = torch.empty_like(self.G)
        kmax, lmax = (K, L) if band is None else (int(band[0]), int(band[1]))
        rad = -1.0 if radius is None else float(radius)
        nb = _step_workspace_size(V, T, K, L, kmax, lmax, rad, _prec(precision))
        self._ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
        self._plan = ctypes.c_void_p()
        vp = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())  # noqa: E731
        check(h.lib.fcfs_pupil_step_plan(
            h.ptr, vp(geom.base_x), vp(geom.base_y), vp(geom.s), vp(geom.hedge), vp(geom.vedge),
            vp(self.offsets), V, T, K, L, kmax, lmax, rad, vp(self.G), vp(self.H),
            _prec(precision), vp(self.loss), vp(self.g_edge), vp(self.F), vp(self._ws),
            ctypes.c_size_t(self._ws.numel()), ctypes.byref(self._plan)), h.ptr)

    def run(self, offsets=None):
        """One step (after copying ``offsets`` in); returns (loss, g_edge)."""
        h = self.handle
        h.sync_stream()
        if offsets is not None:
            self.offsets.copy_(offsets)
        check(h.lib.fcfs_step_plan_launch(h.ptr, self._plan), h.ptr)
        return self.loss, self.g_edge

    def close(self):
        if self._plan:
            self.handle.lib.fcfs_step_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GeneralBatch:
    """Many general tiles (``forward_general`` each) captured once into a
    graph (``fcfs_general_batch_plan``) and replayed by ``run()``.  ``clips``
    holds ``(x, y, s, Nx, Ny, K, L, frac_bits)`` per clip (corners in grid
    units); ``F`` and ``area`` are the plan's output tensors, overwritten by
    every run, which recomputes from the current contents of the corner
    tensors (``corners[i]``).  The plan holds its own workspace."""

    def __init__(self, clips, precision="bf16", handle=None):
        import torch

        h = self.handle = handle or default_handle()
        h.sync_stream()
        dev = h.device
        self.corners, self.F, self.area = [], [], []
        cs = (FcfsGClip * len(clips))()
        for i, (x, y, s, Nx, Ny, K, L, fb) in enumerate(clips):
            x, y, s = _corners_on(dev, x, y, s)
            F = torch.empty((2 * K + 1, 2 * L + 1), dtype=torch.complex64, device=dev)
            a = torch.empty(1, dtype=torch.int64, device=dev)
            self.corners.append((x, y, s))
            self.F.append(F)
            self.area.append(a)
            cs[i] = FcfsGClip(x.data_ptr(), y.data_ptr(), s.data_ptr(), x.numel(), int(Nx),
                              int(Ny), int(fb), int(K), int(L), F.data_ptr(), a.data_ptr())
        self._clips = cs
        nb = ctypes.c_size_t(0)
        check(h.lib.fcfs_general_batch_workspace_size(cs, len(clips), _prec(precision),
                                                      ctypes.byref(nb)))
        self._ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=dev)
        self._plan = ctypes.c_void_p()
        check(h.lib.fcfs_general_batch_plan(h.ptr, cs, len(clips), _prec(precision),
                                            ctypes.c_void_p(self._ws.data_ptr()),
                                            ctypes.c_size_t(self._ws.numel()),
                                            ctypes.byref(self._plan)), h.ptr)

    def run(self):
        """Replays the batch; returns the list of output grids."""
        h = self.handle
        h.sync_stream()
        check(h.lib.fcfs_step_plan_launch(h.ptr, self._plan), h.ptr)
        return self.F

    def close(self):
        if self._plan:
            self.handle.lib.fcfs_step_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@functools.lru_cache(maxsize=64)
def _step_workspace_size(V, T, K, L, kmax, lmax, rad, prec) -> int:
    nb = ctypes.c_size_t(0)
    check(load().fcfs_pupil_step_workspace_size(V, T, K, L, kmax, lmax, rad, prec,
                                                ctypes.byref(nb)))
    return int(nb.value)


@functools.lru_cache(maxsize=1)
def _loss_workspace_size() -> int:
    nb = ctypes.c_size_t(0)
    check(load().fcfs_pupil_loss_workspace_size(ctypes.byref(nb)))
    return int(nb.value)


@functools.lru_cache(maxsize=256)
def _band_workspace_size(V, T, K, L, kmax, lmax, rad, prec) -> int:
    c = _clip(None, None, None, V, T, K, L)
    nb = ctypes.c_size_t(0)
    check(load().fcfs_band_workspace_size(ctypes.byref(c), kmax, lmax, rad, prec, ctypes.byref(nb)))
    return int(nb.value)


def _autograd_function():
    import torch

    class FCFSFunction(torch.autograd.Function):
        """F = FCFS(geometry moved by edge offsets: integers on a square tile,
        multiples of 2^-frac_bits on a general one); backward runs the
        adjoint kernels and the edge reduction.  With ``band`` and/or
        ``radius`` the forward returns the low-pass spectrum (zero outside
        |k| <= kmax, |l| <= lmax, k^2 + l^2 <= radius^2) and the backward is
        its exact adjoint."""

        @staticmethod
        def forward(ctx, offsets, geom, precision="bf16", band=None, radius=None):
            x, y = geom.corners(offsets)
            if geom.general:
                F, _ = forward_general(x, y, geom.s, geom.T, geom.Ny, geom.K, geom.L,
                                       frac_bits=geom.frac_bits, precision=precision,
                                       handle=geom.handle, band=band, radius=radius)
            else:
                F, _ = forward(x, y, geom.s, geom.T, geom.K, geom.L, precision=precision,
                               handle=geom.handle, band=band, radius=radius)
            ctx.geom, ctx.precision, ctx.band, ctx.radius = geom, precision, band, radius
            ctx.save_for_backward(x, y)
            return F

        @staticmethod
        def backward(ctx, grad_F):
            x, y = ctx.saved_tensors
            g = ctx.geom
            if g.general:
                gx, gy = adjoint_general(x, y, g.s, g.T, g.Ny, g.K, g.L, grad_F.contiguous(),
                                         frac_bits=g.frac_bits, precision=ctx.precision,
                                         band=ctx.band, radius=ctx.radius, handle=g.handle)
            else:
                gx, gy = adjoint(x, y, g.s, g.T, g.K, g.L, grad_F.contiguous(), ctx.precision,
                                 band=ctx.band, handle=g.handle, radius=ctx.radius)
            ge = edge_grad(gx, gy, g.hedge, g.vedge, g.n_edges, handle=g.handle)
            return ge, None, None, None, None

    class PupilLoss(torch.autograd.Function):
        """loss = sum |H F - G|^2 (``fcfs_pupil_loss``), H the indicator of the
        disc k^2 + l^2 <= radius^2 (radius None: 1) or the real weights ``H``;
        one kernel computes the value (FP64, fixed order) and the cotangent
        2 H (H F - G) that the backward returns."""

        @staticmethod
        def forward(ctx, F, G, radius=None, H=None, handle=None):
            h = handle or default_handle()
            h.sync_stream()
            F = F.detach().contiguous()
            G = _on(h.device, G, torch.complex64)
            K2, L2 = F.shape
            grad = torch.empty_like(F)
            loss = torch.empty((), dtype=torch.float64, device=h.device)
            Hc = None if H is None else _on(h.device, H, torch.float32)
            ws = h.workspace(_loss_workspace_size())
            check(h.lib.fcfs_pupil_loss(
                h.ptr, ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                None if Hc is None else ctypes.c_void_p(Hc.data_ptr()), (K2 - 1) // 2, (L2 - 1) // 2,
                -1.0 if radius is None else float(radius), ctypes.c_void_p(loss.data_ptr()),
                ctypes.c_void_p(grad.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                ctypes.c_size_t(ws.numel())), h.ptr)
            ctx.save_for_backward(grad)
            return loss

        @staticmethod
        def backward(ctx, grad_out):
            (grad,) = ctx.saved_tensors
            return grad * grad_out.to(grad.real.dtype), None, None, None, None

    return FCFSFunction, PupilLoss


def __getattr__(name):
    if name in ("FCFSFunction", "PupilLoss"):
        f, pl = _autograd_function()
        globals()["FCFSFunction"] = f
        globals()["PupilLoss"] = pl
        return globals()[name]
    raise AttributeError(name)


BATCH_KBUCKET_MAX = (63, 127, 255, 511)


def batch_kbucket(K, L):
    """K bucket of a batch clip (the library's batch_kbucket): the index of the
    first bound in BATCH_KBUCKET_MAX that max(K, L) does not exceed, else 4."""
    m = max(int(K), int(L))
    for i, b in enumerate(BATCH_KBUCKET_MAX):
        if m <= b:
            return i
    return len(BATCH_KBUCKET_MAX)


class Batch:
    """Many clips in one persistent, graph-captured launch (fcfs_forward_batch).

    ``clips``: sequence of (x, y, s, T, K, L) with host or device corner
    arrays.  Inputs are copied to device tensors owned by this object, so the
    captured graph's pointers stay valid; ``run()`` replays it.  Outputs:
    ``F[i]`` ((2K_i+1, 2L_i+1) complex64) and ``area[i]``.  ``tune=True`` runs
    the batch autotuner on these clips first (fcfs_autotune_batch); ``choice``
    maps each K bucket present (``batch_kbucket``) to the (tile variant,
    corners per work item) the plan uses for its clips.
    """

    def __init__(self, clips, precision="bf16", handle=None, tune=False, tune_effort=0):
        import torch

        self.handle = h = handle or default_handle()
        self.precision = _prec(precision)
        dev = h.device
        self.inputs, self.F, self.area = [], [], []
        arr = (FcfsClip * max(1, len(clips)))()
        for i, (x, y, s, T, K, L) in enumerate(clips):
            x, y, s = _corners_on(dev, x, y, s)
            F = torch.empty((2 * K + 1, 2 * L + 1), dtype=torch.complex64, device=dev)
            a = torch.empty(1, dtype=torch.int64, device=dev)
            self.inputs.append((x, y, s))
            self.F.append(F)
            self.area.append(a)
            arr[i] = _clip(x, y, s, x.numel(), T, K, L, F, a)
        self.n = len(clips)
        self._arr = arr
        if tune:
            check(h.lib.fcfs_autotune_batch(h.ptr, arr, self.n, self.precision, int(tune_effort)),
                  h.ptr)
        self.choice = {}
        for kb in sorted({batch_kbucket(c[4], c[5]) for c in clips}):
            tile, chunk = ctypes.c_int32(0), ctypes.c_int64(0)
            check(h.lib.fcfs_batch_choice(h.ptr, self.precision, kb, ctypes.byref(tile),
                                          ctypes.byref(chunk)), h.ptr)
            self.choice[kb] = (int(tile.value), int(chunk.value))
        nb = ctypes.c_size_t(0)
        check(h.lib.fcfs_batch_workspace_size(h.ptr, arr, self.n, self.precision,
                                              ctypes.byref(nb)), h.ptr)
        self.ws = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=dev)
        self._plan = ctypes.c_void_p()

    def run(self):
        h = self.handle
        h.sync_stream()
        check(h.lib.fcfs_forward_batch(h.ptr, self._arr, self.n, self.precision,
                                       ctypes.c_void_p(self.ws.data_ptr()),
                                       ctypes.c_size_t(self.ws.numel()), ctypes.byref(self._plan)),
              h.ptr)
        return self.F

    def close(self):
        if self._plan:
            self.handle.lib.fcfs_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(cache_path=None, effort: int = 1, handle=None):
    """Runs the library's autotuner on this handle (and writes the JSON cache)."""
    h = handle or default_handle()
    h.sync_stream()
    path = None if cache_path is None else str(cache_path).encode()
    check(h.lib.fcfs_autotune(h.ptr, path, int(effort)), h.ptr)


def load_tune(cache_path, handle=None):
    h = handle or default_handle()
    check(h.lib.fcfs_load_tune(h.ptr, str(cache_path).encode()), h.ptr)
