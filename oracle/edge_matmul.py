"""Full coefficient grids of the continuous Fourier series, FP64, with the
general term of Prop. 3 written as one complex matrix product.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library and imports nothing from it.

Same closed forms and the same edge form as ``fcfs_oracle.c`` (Prop. 3 of
Sec. III-C1 for a T x T tile, Sec. II-C basis), for lattice polygons:

    F[0,0] = (1/T)             sum_h  y (x_b - x_a)
    F[k,0] = (j/(2 pi k))      sum_v  (y_a - y_b) e(k x)
    F[0,l] = (j/(2 pi l))      sum_h  (x_b - x_a) e(l y)
    F[k,l] = (-T/(4 pi^2 k l)) sum_h  (e(k x_b) - e(k x_a)) e(l y)

with e(t) = exp(-j 2 pi t / T), h the horizontal edges a -> b at height y and
v the vertical edges a -> b at abscissa x.  The double sum of the general term
is the product D E^T of D[k, h] = e(k x_b) - e(k x_a) and E[l, h] = e(l y_h)
over all horizontal edges: numpy's matrix product does that one step, which
lets a test compare the whole (2K+1) x (2L+1) grid of a 200,000-corner clip
in seconds.  Phases (k x) mod T are reduced exactly in int64 before the
cosine and sine of 2 pi r / T are looked up.  A loop with a negative
edge-form area (counter-clockwise, against the clockwise order of Sec. II-A2)
is counted with the opposite sign, which is the same as reversing it.
"""
from __future__ import annotations

import numpy as np


class EdgeFormError(ValueError):
    pass


def _edges(xy, off):
    """Edges (a -> next vertex of the loop) and the orientation sign of each
    edge's loop; validates that every loop is rectilinear and alternating."""
    xy = np.asarray(xy)
    if xy.size and not np.array_equal(xy, np.round(xy)):
        raise EdgeFormError("lattice coordinates expected")
    xy = np.asarray(xy, dtype=np.int64).reshape(-1, 2)
    off = np.asarray(off, dtype=np.int64).ravel()
    if off.size < 1 or off[0] != 0 or off[-1] != xy.shape[0] or np.any(np.diff(off) < 0):
        raise EdgeFormError("loop offsets do not match the vertex array")
    n = xy.shape[0]
    cnt = np.diff(off)
    if np.any(cnt < 4) or np.any(cnt % 2):
        raise EdgeFormError("every loop needs an even number (>= 4) of vertices")
    loop = np.repeat(np.arange(cnt.size), cnt)
    a = np.arange(n)
    b = np.where(a + 1 == off[loop + 1], off[loop], a + 1)
    xa, ya, xb, yb = xy[a, 0], xy[a, 1], xy[b, 0], xy[b, 1]
    hor = (ya == yb) & (xa != xb)
    ver = (xa == xb) & (ya != yb)
    if not np.all(hor | ver):
        raise EdgeFormError("an edge is neither horizontal nor vertical")
    # edges alternate: edge a and edge b (the next one) have different kinds
    if np.any(hor == hor[b]):
        raise EdgeFormError("edges do not alternate")
    la = np.zeros(cnt.size, dtype=np.int64)
    np.add.at(la, loop[hor], ya[hor] * (xb[hor] - xa[hor]))
    if np.any(la == 0):
        raise EdgeFormError("a loop has zero area")
    sigma = np.where(la > 0, 1, -1)[loop]
    return xa, ya, xb, yb, hor, sigma, int(np.sum(np.abs(la)))


def cfs_grid_matmul(xy, off, T: int, K: int, L: int):
    """Coefficients F[k, l], |k| <= K, |l| <= L, of lattice polygon loops over a
    T x T tile: a (2K+1, 2L+1) complex128 array indexed [k + K, l + L], and
    the exact integer area (a Python int)."""
    T, K, L = int(T), int(K), int(L)
    if T < 1 or K < 0 or L < 0:
        raise EdgeFormError("T >= 1 and K, L >= 0 expected")
    xa, ya, xb, yb, hor, sigma, _ = _edges(xy, off)
    ver = ~hor
    p = np.arange(T, dtype=np.float64)
    ang = 2.0 * np.pi * p / T
    w = np.cos(ang) - 1j * np.sin(ang)  # e(p) for p = 0 .. T-1
    k = np.arange(-K, K + 1, dtype=np.int64)
    l = np.arange(-L, L + 1, dtype=np.int64)
    F = np.zeros((2 * K + 1, 2 * L + 1), dtype=np.complex128)

    sh = sigma[hor].astype(np.float64)
    hxa, hxb, hy = xa[hor], xb[hor], ya[hor]
    area = int(np.sum(sigma[hor] * hy * (hxb - hxa)))
    F[K, L] = area / T

    # general term: D[k, h] E[l, h] summed over the horizontal edges
    D = w[(k[:, None] * hxb[None, :]) % T]
    D -= w[(k[:, None] * hxa[None, :]) % T]
    D *= sh[None, :]
    E = w[(l[:, None] * hy[None, :]) % T]
    S = D @ E.T
    del D, E
    kk, ll = np.meshgrid(k.astype(np.float64), l.astype(np.float64), indexing="ij")
    gen = (kk != 0) & (ll != 0)
    F[gen] = -T / (4.0 * np.pi ** 2 * kk[gen] * ll[gen]) * S[gen]

    # F[k, 0]: vertical edges a -> b at x
    sv = (sigma[ver] * (ya[ver] - yb[ver])).astype(np.float64)
    vx = xa[ver]
    nz = k != 0
    Fk = w[(k[nz, None] * vx[None, :]) % T] @ sv
    F[nz, L] = 1j / (2.0 * np.pi * k[nz]) * Fk
    # F[0, l]: horizontal edges a -> b at y
    sx = (sigma[hor] * (hxb - hxa)).astype(np.float64)
    nz = l != 0
    Fl = w[(l[nz, None] * hy[None, :]) % T] @ sx
    F[K, nz] = 1j / (2.0 * np.pi * l[nz]) * Fl
    return F, area
