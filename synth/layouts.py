"""Seeded generators of rectilinear layout clips.

Recipe (the paper's layouts are proprietary; these stand in for them):

* a polygon is the union of ``n ~ U{1..10}`` rectangles with widths and heights
  ``~ U{20..400}``; rectangle ``i > 0`` is placed so that it overlaps a random
  earlier one with positive area, so the union is connected;
* the union's boundary is traced on the compressed coordinate grid; a union
  with a hole, a saddle point (two cells touching at one corner only) or a
  vertex count outside ``[4, 40]`` is redrawn;
* the polygon is translated uniformly so that its bounding box lies in
  ``[0, T]^2`` (redrawn if it does not fit);
* loops are emitted clockwise, polygon after polygon, never sorted.

``disjoint=True`` confines each polygon to its own cell of a jittered grid and
scales rectangle sizes to the cell, so polygons never overlap (fill factor of
the clip well below one, as in a real layer).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Clip:
    """One clip: polygon loops plus the tile period and cut-offs it is meant for."""

    xy: np.ndarray  # (n_vertices, 2) int32
    off: np.ndarray  # (n_loops + 1,) int64
    T: int
    K: int
    L: int
    seed: int

    @property
    def n_vertices(self) -> int:
        return int(self.off[-1])

    @property
    def n_loops(self) -> int:
        return int(self.off.size - 1)


def rectangle_loop(x1: int, y1: int, x2: int, y2: int) -> np.ndarray:
    """Clockwise loop (y up) of the half-open rectangle [x1,x2) x [y1,y2)."""
    return np.array([[x1, y1], [x1, y2], [x2, y2], [x2, y1]], dtype=np.int32)


def _occupancy(rects: np.ndarray):
    xs = np.unique(np.concatenate([rects[:, 0], rects[:, 2]]))
    ys = np.unique(np.concatenate([rects[:, 1], rects[:, 3]]))
    # occ[i, j] = 1 if the cell [xs[i-1], xs[i]) x [ys[j-1], ys[j]) is covered
    occ = np.zeros((xs.size + 1, ys.size + 1), dtype=np.int8)
    i1 = np.searchsorted(xs, rects[:, 0])
    i2 = np.searchsorted(xs, rects[:, 2])
    j1 = np.searchsorted(ys, rects[:, 1])
    j2 = np.searchsorted(ys, rects[:, 3])
    for a, b, c, d in zip(i1, i2, j1, j2):
        occ[a + 1 : b + 1, c + 1 : d + 1] = 1
    return xs, ys, occ


def loops_of_rect_union(rects) -> list[np.ndarray] | None:
    """Boundary loops of the union of rectangles ``(x1, y1, x2, y2)``.

    Returns the loops (each an ``(n, 2)`` int32 array, clockwise when it bounds
    a covered region from outside), or None when the union has a saddle point
    (where the boundary would touch itself).
    """
    rects = np.asarray(rects, dtype=np.int64).reshape(-1, 4)
    if rects.size == 0:
        return []
    if np.any(rects[:, 2] <= rects[:, 0]) or np.any(rects[:, 3] <= rects[:, 1]):
        raise ValueError("empty rectangle")
    xs, ys, occ = _occupancy(rects)
    # Grid point (i, j) sits at (xs[i], ys[j]); the four cells around it are
    # occ[i..i+1, j..j+1].  It is a corner of the boundary when an odd number
    # of them is covered, a saddle when exactly the two diagonal ones are.
    a = occ[:-1, :-1].astype(np.int32)  # lower-left cell
    b = occ[1:, :-1].astype(np.int32)   # lower-right
    c = occ[:-1, 1:].astype(np.int32)   # upper-left
    d = occ[1:, 1:].astype(np.int32)    # upper-right
    cnt = a + b + c + d
    saddle = (cnt == 2) & (a == d)
    if np.any(saddle):
        return None
    ci, cj = np.nonzero(cnt % 2 == 1)
    n = ci.size
    if n == 0:
        return []
    # Link corners along each horizontal line (same j) and each vertical line
    # (same i): sorted along the line, consecutive pairs bound one edge.
    hpart = np.empty(n, dtype=np.int64)
    vpart = np.empty(n, dtype=np.int64)
    order = np.lexsort((ci, cj))  # by j, then i
    for k in range(0, n, 2):
        p, q = order[k], order[k + 1]
        hpart[p], hpart[q] = q, p
    order = np.lexsort((cj, ci))  # by i, then j
    for k in range(0, n, 2):
        p, q = order[k], order[k + 1]
        vpart[p], vpart[q] = q, p
    seen = np.zeros(n, dtype=bool)
    loops = []
    for start in range(n):
        if seen[start]:
            continue
        seq = []
        cur, horiz = start, True
        while True:
            seen[cur] = True
            seq.append(cur)
            cur = hpart[cur] if horiz else vpart[cur]
            horiz = not horiz
            if cur == start:
                break
        pts = np.stack([xs[ci[seq]], ys[cj[seq]]], axis=1)
        # orientation from the horizontal edges: sum y (x_next - x) > 0 when clockwise
        nxt = np.roll(pts, -1, axis=0)
        hmask = pts[:, 1] == nxt[:, 1]
        area = int(np.sum(pts[hmask, 1] * (nxt[hmask, 0] - pts[hmask, 0])))
        if area < 0:
            pts = pts[::-1]
        loops.append(pts.astype(np.int32))
    return loops


def _one_polygon(rng: np.random.Generator, lo: int, hi: int, vmax: int,
                 box: tuple[int, int] | None):
    """Draw rectangles until their union is one simple loop with <= vmax
    vertices whose bounding box fits in ``box`` (width, height)."""
    while True:
        n = int(rng.integers(1, 11))
        r = np.zeros((n, 4), dtype=np.int64)
        w = rng.integers(lo, hi + 1, size=n)
        h = rng.integers(lo, hi + 1, size=n)
        r[0] = (0, 0, w[0], h[0])
        for i in range(1, n):
            j = int(rng.integers(0, i))
            x1 = int(rng.integers(r[j, 0] - w[i] + 1, r[j, 2]))
            y1 = int(rng.integers(r[j, 1] - h[i] + 1, r[j, 3]))
            r[i] = (x1, y1, x1 + w[i], y1 + h[i])
        loops = loops_of_rect_union(r)
        if loops is None or len(loops) != 1:
            continue
        p = loops[0]
        if p.shape[0] > vmax:
            continue
        p = p.astype(np.int64)
        p -= p.min(axis=0)
        if box is not None:
            bw, bh = int(p[:, 0].max()), int(p[:, 1].max())
            if bw > box[0] or bh > box[1]:
                continue
        return p


def _pack(loops: list[np.ndarray]):
    off = np.zeros(len(loops) + 1, dtype=np.int64)
    off[1:] = np.cumsum([p.shape[0] for p in loops])
    xy = np.concatenate(loops, axis=0).astype(np.int32) if loops else np.zeros((0, 2), np.int32)
    return xy, off


def clip(seed: int, T: int, K: int, L: int | None = None, *, n_polygons: int | None = None,
         min_vertices: int | None = None, disjoint: bool = False,
         size_scale: float = 1.0) -> Clip:
    """A clip of random polygons (see the module docstring for the recipe).

    Exactly one of ``n_polygons`` (a fixed count) or ``min_vertices`` (draw
    polygons until the total vertex count reaches it) must be given.
    ``size_scale`` (disjoint clips only) multiplies the rectangle sizes drawn
    for a cell (cell/20 .. cell/4 at 1.0), which sets the fill factor.
    """
    if (n_polygons is None) == (min_vertices is None):
        raise ValueError("give n_polygons or min_vertices")
    L = K if L is None else L
    rng = np.random.default_rng(np.random.PCG64(seed))
    loops = []
    total = 0
    if not disjoint:
        def more():
            return len(loops) < n_polygons if n_polygons is not None else total < min_vertices
        while more():
            p = _one_polygon(rng, 20, 400, 40, (T, T))
            bw, bh = int(p[:, 0].max()), int(p[:, 1].max())
            dx = int(rng.integers(0, T - bw + 1))
            dy = int(rng.integers(0, T - bh + 1))
            p = p + np.array([dx, dy])
            loops.append(p)
            total += p.shape[0]
    else:
        # Estimate the polygon count, then give each polygon its own cell.
        # (larger rectangles make simpler unions: fewer corners per polygon)
        per = 14.0 if size_scale == 1.0 else 8.0
        want = n_polygons if n_polygons is not None else int(np.ceil(min_vertices / per)) + 16
        g = int(np.ceil(np.sqrt(want)))
        cell = T // g
        if cell < 16:
            raise ValueError("too many polygons for disjoint cells")
        lo = max(2, int(cell * size_scale) // 20)
        hi = min(cell - 2, max(lo + 1, int(cell * size_scale) // 4))
        cells = rng.permutation(g * g)
        for c in cells:
            if n_polygons is not None and len(loops) >= n_polygons:
                break
            if n_polygons is None and total >= min_vertices:
                break
            p = _one_polygon(rng, lo, hi, 40, (cell - 2, cell - 2))
            bw, bh = int(p[:, 0].max()), int(p[:, 1].max())
            cx, cy = (int(c) % g) * cell, (int(c) // g) * cell
            dx = cx + 1 + int(rng.integers(0, cell - 2 - bw + 1))
            dy = cy + 1 + int(rng.integers(0, cell - 2 - bh + 1))
            p = p + np.array([dx, dy])
            loops.append(p)
            total += p.shape[0]
        if n_polygons is None and total < min_vertices:
            raise ValueError("disjoint grid too small for the requested vertex count")
    xy, off = _pack(loops)
    return Clip(xy, off, int(T), int(K), int(L), int(seed))


def clip_c1(seed: int = 1, T: int = 2048, K: int = 64, n_vertices: int = 64,
            min_rects: int = 8, max_rects: int = 32) -> tuple[Clip, int, int]:
    """One polygon built as a union of rectangles with corners uniform in [0, T).

    Rectangles are drawn one after another from sub-seed ``seed``; from the
    ``min_rects``-th on, the first union that is one simple loop with exactly
    ``n_vertices`` corners is returned.  After ``max_rects`` rectangles the
    next sub-seed starts over.  Returns ``(clip, sub_seed, n_rects)``.
    """
    sub = seed
    while True:
        rng = np.random.default_rng(np.random.PCG64(sub))
        rects = []
        for nr in range(1, max_rects + 1):
            while True:
                a = rng.integers(0, T, size=4)
                x1, x2 = sorted((int(a[0]), int(a[2])))
                y1, y2 = sorted((int(a[1]), int(a[3])))
                if x1 < x2 and y1 < y2:
                    break
            rects.append((x1, y1, x2, y2))
            if nr < min_rects:
                continue
            loops = loops_of_rect_union(rects)
            if loops is not None and len(loops) == 1 and loops[0].shape[0] == n_vertices:
                xy, off = _pack(loops)
                return Clip(xy, off, T, K, K, seed), sub, nr
        sub += 1


def shift_loops(xy: np.ndarray, dx: int, dy: int) -> np.ndarray:
    """Translate every vertex by (dx, dy)."""
    out = np.asarray(xy).astype(np.int64) + np.array([dx, dy], dtype=np.int64)
    return out.astype(np.int32)


# (T, K) pairs of the batched form: the cut-off grows with the period.
BATCH_TK = ((1024, 63), (2048, 127), (4096, 255), (8192, 511))


def batch_clips(seed: int, n_clips: int = 256, v_lo: int = 1000, v_hi: int = 200_000,
                pool: int = 4096) -> list[Clip]:
    """Clips of the batched form: vertex counts log-uniform in [v_lo, v_hi],
    (T, K) drawn uniformly from ``BATCH_TK``.

    To keep generation fast at millions of vertices, every clip draws its
    polygons (with replacement) from one seeded pool of ``pool`` shapes made
    by the same polygon recipe, each placed at a uniform random offset.
    """
    rng = np.random.default_rng(np.random.PCG64(seed))
    shapes = [_one_polygon(rng, 20, 400, 40, (1024, 1024)) for _ in range(pool)]
    sizes = np.array([s.shape[0] for s in shapes], dtype=np.int64)
    ext = np.array([s.max(axis=0) for s in shapes], dtype=np.int64)
    out = []
    for c in range(n_clips):
        T, K = BATCH_TK[int(rng.integers(0, len(BATCH_TK)))]
        vt = int(np.exp(rng.uniform(np.log(v_lo), np.log(v_hi))))
        # pick shapes until the vertex target is met
        ids = []
        tot = 0
        while tot < vt:
            chunk = rng.integers(0, pool, size=max(16, (vt - tot) // 12))
            for i in chunk:
                ids.append(int(i))
                tot += int(sizes[i])
                if tot >= vt:
                    break
        ids = np.array(ids, dtype=np.int64)
        dx = (rng.random(ids.size) * (T - ext[ids, 0] + 1)).astype(np.int64)
        dy = (rng.random(ids.size) * (T - ext[ids, 1] + 1)).astype(np.int64)
        loops = [shapes[i] + np.array([a, b]) for i, a, b in zip(ids, dx, dy)]
        xy, off = _pack(loops)
        out.append(Clip(xy, off, T, K, K, seed * 1000 + c))
    return out
