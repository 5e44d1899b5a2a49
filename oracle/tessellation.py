"""Oracle: the overlapping-subarray tessellation of Section II-D (test
infrastructure only).

The array is cut into hexagonal cells; each cell has an inner, non-overlapping
part of radius R_in and an extended part out to R_in + R_ext.  Every cell's
subarray (all antennas within the outer hexagon) is analysed on its own, and
only the results of the antennas of the inner part are kept (subarray figure,
Section II-D; Section IV-B).

Readings (the paper gives no coordinates or orientation):
* the inner parts are the regular flat-top hexagons (two vertices on the x axis)
  of circumradius R_in that tile the plane, centred on the lattice
  o + (1.5 R_in i, sqrt(3) R_in (j + i/2)); an antenna belongs to the hexagon
  containing it, i.e. to the nearest centre (ties: the smallest (i, j));
* the outer part is the concentric flat-top hexagon of circumradius R_in + R_ext;
* the subarray is solved with the same fill and dense solve as a whole layout
  (the radius of influence is the subarray itself), with a unit voltage at each
  inner antenna's port; the subarray lists its inner antennas first, then the
  others, each in ascending index order.

Written independently of the library: the nearest centre is found by brute
force over every centre covering the layout's bounding box, and membership of a
hexagon by the six half-planes of its edges.
"""
from __future__ import annotations

import math

import numpy as np

from . import fill as ofill, patterns as opat, solve as osolve
from .fit import Model


def hexagon_vertices(cx: float, cy: float, radius: float) -> np.ndarray:
    """Flat-top hexagon: vertices at angles 0, 60, ..., 300 degrees."""
    a = np.arange(6) * (math.pi / 3.0)
    return np.stack([cx + radius * np.cos(a), cy + radius * np.sin(a)], axis=1)


def in_hexagon(px, py, verts: np.ndarray) -> np.ndarray:
    """Points inside or on the convex hexagon (counter-clockwise vertices):
    on the left of, or on, every directed edge."""
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    inside = np.ones(px.shape, dtype=bool)
    for k in range(6):
        (x0, y0), (x1, y1) = verts[k], verts[(k + 1) % 6]
        cross = (x1 - x0) * (py - y0) - (y1 - y0) * (px - x0)
        inside &= cross >= -1e-12 * max(1.0, abs(x1 - x0) + abs(y1 - y0))
    return inside


def lattice_centres(x, y, r_in: float, origin=(0.0, 0.0)):
    """Every lattice centre (i, j, cx, cy) whose cell can touch the layout's
    bounding box (with one cell of margin), sorted by (i, j)."""
    ox, oy = origin
    i_lo = math.floor((np.min(x) - ox) / (1.5 * r_in)) - 2
    i_hi = math.ceil((np.max(x) - ox) / (1.5 * r_in)) + 2
    out = []
    for i in range(i_lo, i_hi + 1):
        # cy = oy + sqrt(3) r (j + i/2) must span [min y, max y] with margin
        j_lo = math.floor((np.min(y) - oy) / (math.sqrt(3.0) * r_in) - i / 2.0) - 2
        j_hi = math.ceil((np.max(y) - oy) / (math.sqrt(3.0) * r_in) - i / 2.0) + 2
        for j in range(j_lo, j_hi + 1):
            out.append((i, j, ox + 1.5 * r_in * i, oy + math.sqrt(3.0) * r_in * (j + 0.5 * i)))
    return out


def tessellate(x, y, r_in: float, r_ext: float, origin=(0.0, 0.0)):
    """List of (centre (cx, cy), members with the inner antennas first, number
    of inner antennas), one per cell with at least one inner antenna, in (i, j)
    order."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    cen = lattice_centres(x, y, r_in, origin)
    C = np.array([[c[2], c[3]] for c in cen])
    d2 = (x[:, None] - C[None, :, 0]) ** 2 + (y[:, None] - C[None, :, 1]) ** 2
    own = np.argmin(d2, axis=1)            # first minimum = smallest (i, j)
    cells = []
    for k in sorted(set(own.tolist())):
        cx, cy = C[k]
        inner = np.flatnonzero(own == k)
        outer = in_hexagon(x, y, hexagon_vertices(cx, cy, r_in + r_ext))
        others = np.flatnonzero(outer & (own != k))
        cells.append(((float(cx), float(cy)), np.concatenate([inner, others]), int(inner.size)))
    return cells


def solve_tessellated(model: Model, x, y, r_in: float, r_ext: float, theta=None, phi=None, origin=(0.0, 0.0)):
    """Per antenna a: (subarray members, X column, Y column) of a unit voltage at
    its port from its own cell's subarray, and, if directions are given, the
    embedded element patterns E[a, dir, (theta, phi)] over that subarray."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    out = [None] * x.size
    E = None if theta is None else np.zeros((x.size, np.size(theta), 2), dtype=np.complex128)
    for _, mem, ni in tessellate(x, y, r_in, r_ext, origin):
        xs, ys = x[mem], y[mem]
        Z = ofill.fill(model, xs, ys)
        B = osolve.port_rhs(model.w, mem.size)[:, :ni]
        X = osolve.solve(Z, B)
        Y = osolve.admittance(X, model.w, mem.size)
        for k in range(ni):
            out[mem[k]] = (mem, X[:, k], Y[:, k])
        if E is not None:
            E[mem[:ni]] = opat.embedded_patterns(model.freq, model.samples, xs, ys, X, theta, phi)
    return out, E
