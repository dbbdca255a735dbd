"""Independent reference quantities used to pin the oracle (test code only).

Nothing here calls the oracle or the HIP library; every function is an
independent route to a value the CFS must equal.
"""
from __future__ import annotations

import numpy as np


def rect_cfs(x1, y1, x2, y2, T, K, L):
    """CFS of the rectangle [x1,x2) x [y1,y2) by direct integration of the
    orthonormal Fourier basis (Sec. II-C): a product of two sinc factors."""
    k = np.arange(-K, K + 1)[:, None].astype(np.float64)
    l = np.arange(-L, L + 1)[None, :].astype(np.float64)
    dx, dy = x2 - x1, y2 - y1
    ph = np.exp(-1j * np.pi * (k * (x1 + x2) + l * (y1 + y2)) / T)
    return dx * dy / T * ph * np.sinc(k * dx / T) * np.sinc(l * dy / T)


def rect_interval(a, b, f, T):
    """integral_a^b e^{-j 2 pi f t / T} dt for an integer array f (f = 0 -> b - a)."""
    f = np.asarray(f, dtype=np.float64)
    return (b - a) * np.exp(-1j * np.pi * f * (a + b) / T) * np.sinc(f * (b - a) / T)


def raster(xy, off, T):
    """Cell occupancy count image (T x T, cell (i, j) = [i,i+1) x [j,j+1)) of
    loops whose coordinates lie in [0, T], by scanline even-odd filling."""
    img = np.zeros((T, T), dtype=np.int64)
    xy = np.asarray(xy, dtype=np.int64)
    for m in range(len(off) - 1):
        p = xy[off[m]:off[m + 1]]
        q = np.roll(p, -1, axis=0)
        one = np.zeros((T, T), dtype=np.int64)
        # vertical edges toggle the cells to their right (even-odd rule)
        for (xa, ya), (xb, yb) in zip(p, q):
            if xa == xb:
                lo, hi = min(ya, yb), max(ya, yb)
                one[xa:, lo:hi] ^= 1
        img += one
    return img


def raster_cfs(img, T, K, L):
    """Exact CFS of a union of unit lattice cells: each cell integrates to
    (1/T) e^{-j w (k (i+1/2) + l (j+1/2))} sinc(k/T) sinc(l/T)."""
    i = np.arange(T) + 0.5
    k = np.arange(-K, K + 1)
    l = np.arange(-L, L + 1)
    Ek = np.exp(-2j * np.pi * np.outer(k, i) / T)
    El = np.exp(-2j * np.pi * np.outer(l, i) / T)
    S = Ek @ img.astype(np.float64) @ El.T
    return S / T * np.sinc(k / T)[:, None] * np.sinc(l / T)[None, :]


def corner_image(img):
    """Signed corner weights w[x, y] (lattice points) of a cell image: the mixed
    second difference, so that the image equals sum_w w * 1[X >= x, Y >= y]."""
    T = img.shape[0]
    O = np.zeros((T + 1, T + 1), dtype=np.int64)
    O[:T, :T] = img
    W = O.copy()
    W[1:, :] -= O[:-1, :]
    W2 = W.copy()
    W2[:, 1:] -= W[:, :-1]
    return W2


def shoelace2(xy, off):
    """Twice the signed shoelace area of every loop (positive counter-clockwise
    in the usual convention)."""
    xy = np.asarray(xy, dtype=np.int64)
    out = []
    for m in range(len(off) - 1):
        p = xy[off[m]:off[m + 1]]
        q = np.roll(p, -1, axis=0)
        out.append(int(np.sum(p[:, 0] * q[:, 1] - q[:, 0] * p[:, 1])))
    return np.array(out, dtype=np.int64)
