"""Seeded synthetic layout clips (rectilinear polygon loops).

This module is shared by the tests, the benchmark and the smoke check.  It only
draws geometry: rectangles, their unions and their boundary loops.  It computes
nothing of the Fourier method itself (no phases, no coefficients and no corner
signs), so that neither the oracle nor the HIP library depends on the other
through it.

Output format, everywhere: ``(xy, off)`` with ``xy`` an ``(n_vertices, 2)``
int32 array of lattice coordinates and ``off`` an ``(n_loops + 1,)`` int64
array of loop offsets.  Each loop is a simple rectilinear lattice polygon
without holes (Sec. II-A2 of the paper), listed clockwise with y pointing up,
vertices polygon-contiguous and in loop order.
"""
from .layouts import (  # noqa: F401
    Clip,
    batch_clips,
    clip,
    clip_c1,
    loops_of_rect_union,
    rectangle_loop,
    shift_loops,
)
