"""CPU oracles for the continuous Fourier series (FP64) and the pruned
continuous Haar transform (exact integer areas) of rectilinear polygons.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library (``paper_1010_5562_amd``) and imports nothing from it.

The arithmetic lives in ``fcfs_oracle.c`` (plain C, FP64, optional OpenMP)
and ``pcht_oracle.c`` (plain C, int64 areas); this module only compiles them
with gcc and marshals numpy arrays through ctypes.  ``edge_matmul.py`` holds
the same edge form in numpy with the general term as one matrix product
(``cfs_grid_matmul``), for full grids of large clips.  See the headers of the C
files for the formulas and their sources in the paper (Prop. 3 of Sec.
III-C1, edge form; Sec. III-B1 and Algorithm 1 for the Haar transform).

Polygons are passed as loops: ``xy`` is an ``(n_vertices, 2)`` array of
coordinates, ``off`` an ``(n_loops + 1,)`` int64 array of loop offsets.  Edge
``e`` joins vertex ``e`` to the next vertex of its loop.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .edge_matmul import EdgeFormError, cfs_grid_matmul  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "fcfs_oracle.c"), os.path.join(_HERE, "pcht_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle_fcfs.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-fopenmp", "-Wall", "-shared", "-fPIC", *_SRCS, "-o", tmp, "-lm"],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32, c_int = ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    lib.fo_cfs_grid.argtypes = [P, P, i64, i64, i32, i32, c_int, c_int, P, P]
    lib.fo_cfs_points.argtypes = [P, P, i64, i64, c_int, i64, P, P, c_int, P]
    lib.fo_edge_grad.argtypes = [P, P, i64, i64, i32, i32, c_int, P, P, i64, c_int, P]
    lib.fo_loop_areas.argtypes = [P, P, i64, P]
    lib.fo_threads.argtypes = [c_int]
    lib.po_pcht.argtypes = [P, P, i64, i64, i64, c_int, P, P, P]
    lib.fo_cfs_grid_general.argtypes = [P, P, i64, i64, i64, i32, i32, i32, c_int, P, P]
    lib.fo_cfs_grid_general.restype = ctypes.c_int
    lib.fo_cfs_points_general.argtypes = [P, P, i64, i64, i64, i32, i64, P, P, c_int, P]
    lib.fo_cfs_points_general.restype = ctypes.c_int
    lib.fo_edge_grad_general.argtypes = [P, P, i64, i64, i64, i32, i32, i32, P, P, i64, c_int, P]
    lib.fo_edge_grad_general.restype = ctypes.c_int
    lib.po_pcht.restype = ctypes.c_int
    for f in (lib.fo_cfs_grid, lib.fo_cfs_points, lib.fo_edge_grad, lib.fo_loop_areas,
              lib.fo_threads):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _loops(xy, off):
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64).reshape(-1, 2))
    off = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    if off.ndim != 1 or off.size < 1 or off[-1] != xy.shape[0]:
        raise OracleError("loop offsets do not match the vertex array")
    return xy, off


def _check(st, what):
    if st != 0:
        raise OracleError(f"{what} failed with status {st}")


def threads(n: int = 0) -> int:
    """Set (n > 0) and report the OpenMP thread count the oracle uses."""
    return int(_load().fo_threads(int(n)))


def cfs_grid(xy, off, T: int, K: int, L: int, lattice: bool = True, nthreads: int = 0):
    """Coefficients F[k, l] for |k| <= K, |l| <= L as a (2K+1, 2L+1) complex128
    array indexed [k + K, l + L], and the exact integer area (lattice mode)."""
    lib = _load()
    xy, off = _loops(xy, off)
    F = np.zeros((2 * K + 1) * (2 * L + 1) * 2, dtype=np.float64)
    area = np.zeros(1, dtype=np.int64)
    st = lib.fo_cfs_grid(_ptr(xy), _ptr(off), off.size - 1, int(T), int(K), int(L),
                         int(bool(lattice)), int(nthreads), _ptr(F), _ptr(area))
    _check(st, "fo_cfs_grid")
    return F.view(np.complex128).reshape(2 * K + 1, 2 * L + 1), int(area[0])


def cfs_grid_general(xy, off, Nx: int, Ny: int, K: int, L: int, frac_bits: int = 0,
                     nthreads: int = 0):
    """Coefficients over an Nx x Ny tile (Prop. 3 with its general factors) for
    vertices on the grid of step 2^-frac_bits (``xy`` holds the true
    coordinates).  Returns ``(F, area)``, F (2K+1, 2L+1) complex128 indexed
    [k + K, l + L] and area = the signed area times 4^frac_bits (exact)."""
    lib = _load()
    xy, off = _loops(xy, off)
    F = np.zeros((2 * K + 1) * (2 * L + 1) * 2, dtype=np.float64)
    area = np.zeros(1, dtype=np.int64)
    st = lib.fo_cfs_grid_general(_ptr(xy), _ptr(off), off.size - 1, int(Nx), int(Ny),
                                 int(frac_bits), int(K), int(L), int(nthreads), _ptr(F),
                                 _ptr(area))
    _check(st, "fo_cfs_grid_general")
    return F.view(np.complex128).reshape(2 * K + 1, 2 * L + 1), int(area[0])


def cfs_points_general(xy, off, Nx: int, Ny: int, k, l, frac_bits: int = 0, nthreads: int = 0):
    """Single coefficients F[k[i], l[i]] of a general tile (as
    ``cfs_grid_general``), a complex128 vector."""
    lib = _load()
    xy, off = _loops(xy, off)
    k = np.ascontiguousarray(np.asarray(k, dtype=np.int32).ravel())
    l = np.ascontiguousarray(np.asarray(l, dtype=np.int32).ravel())
    if k.size != l.size:
        raise OracleError("k and l differ in length")
    F = np.zeros(k.size * 2, dtype=np.float64)
    st = lib.fo_cfs_points_general(_ptr(xy), _ptr(off), off.size - 1, int(Nx), int(Ny),
                                   int(frac_bits), k.size, _ptr(k), _ptr(l), int(nthreads),
                                   _ptr(F))
    _check(st, "fo_cfs_points_general")
    return F.view(np.complex128)


def cfs_points(xy, off, T: int, k, l, lattice: bool = True, nthreads: int = 0):
    """Single coefficients F[k[i], l[i]] as a complex128 vector."""
    lib = _load()
    xy, off = _loops(xy, off)
    k = np.ascontiguousarray(np.asarray(k, dtype=np.int32).ravel())
    l = np.ascontiguousarray(np.asarray(l, dtype=np.int32).ravel())
    if k.size != l.size:
        raise OracleError("k and l differ in length")
    F = np.zeros(k.size * 2, dtype=np.float64)
    st = lib.fo_cfs_points(_ptr(xy), _ptr(off), off.size - 1, int(T), int(bool(lattice)),
                           k.size, _ptr(k), _ptr(l), int(nthreads), _ptr(F))
    _check(st, "fo_cfs_points")
    return F.view(np.complex128)


def edge_grad(xy, off, T: int, K: int, L: int, G, edges=None, lattice: bool = True,
              nthreads: int = 0):
    """dLoss/d(edge offset) for every edge (or the listed ones), given the
    complex cotangent G = dLoss/dRe F + j dLoss/dIm F on the centred grid."""
    lib = _load()
    xy, off = _loops(xy, off)
    G = np.ascontiguousarray(np.asarray(G, dtype=np.complex128).reshape(2 * K + 1, 2 * L + 1))
    Gf = G.view(np.float64).ravel()
    if edges is None:
        n = int(off[-1])
        sel = None
    else:
        sel = np.ascontiguousarray(np.asarray(edges, dtype=np.int64).ravel())
        n = sel.size
    g = np.zeros(max(n, 1), dtype=np.float64)
    st = lib.fo_edge_grad(_ptr(xy), _ptr(off), off.size - 1, int(T), int(K), int(L),
                          int(bool(lattice)), _ptr(Gf), None if sel is None else _ptr(sel),
                          0 if sel is None else sel.size, int(nthreads), _ptr(g))
    _check(st, "fo_edge_grad")
    return g[:n]


def edge_grad_general(xy, off, Nx: int, Ny: int, K: int, L: int, G, frac_bits: int = 0,
                      edges=None, nthreads: int = 0):
    """dLoss/d(edge offset), true units, for a general tile; as ``edge_grad``."""
    lib = _load()
    xy, off = _loops(xy, off)
    G = np.ascontiguousarray(np.asarray(G, dtype=np.complex128).reshape(2 * K + 1, 2 * L + 1))
    Gf = G.view(np.float64).ravel()
    if edges is None:
        n = int(off[-1])
        sel = None
    else:
        sel = np.ascontiguousarray(np.asarray(edges, dtype=np.int64).ravel())
        n = sel.size
    g = np.zeros(max(n, 1), dtype=np.float64)
    st = lib.fo_edge_grad_general(_ptr(xy), _ptr(off), off.size - 1, int(Nx), int(Ny),
                                  int(frac_bits), int(K), int(L), _ptr(Gf),
                                  None if sel is None else _ptr(sel), 0 if sel is None else sel.size,
                                  int(nthreads), _ptr(g))
    _check(st, "fo_edge_grad_general")
    return g[:n]


def loop_areas(xy, off):
    """Exact signed edge-form area of every loop (positive when clockwise)."""
    lib = _load()
    xy, off = _loops(xy, off)
    a = np.zeros(max(off.size - 1, 1), dtype=np.int64)
    _check(lib.fo_loop_areas(_ptr(xy), _ptr(off), off.size - 1, _ptr(a)), "fo_loop_areas")
    return a[: off.size - 1]


def pcht(xy, off, Nx: int, Ny: int, J: int):
    """Pruned continuous Haar transform of the polygons over [0,Nx) x [0,Ny)
    with J levels of wavelets.  Returns ``(U, W, nodes)``: U the 2^J x 2^J
    int64 pyramid of integer area sums, W the coefficients (float64), nodes
    the number of non-terminating recursive calls."""
    lib = _load()
    xy, off = _loops(xy, off)
    side = 1 << int(J)
    U = np.zeros(side * side, dtype=np.int64)
    W = np.zeros(side * side, dtype=np.float64)
    nodes = np.zeros(1, dtype=np.int64)
    st = lib.po_pcht(_ptr(xy), _ptr(off), off.size - 1, int(Nx), int(Ny), int(J), _ptr(U),
                     _ptr(W), _ptr(nodes))
    _check(st, "po_pcht")
    return U.reshape(side, side), W.reshape(side, side), int(nodes[0])
