"""Sibson natural-neighbour weights on the parent lattice (FP64).

Oracle (test infrastructure).  The paper writes each aperture (detector) beam
as a local convex combination of parent beams using Sibson natural-neighbour
interpolation on signed-frequency coordinates (eq. nnw, section
"Partitioned PRISM-EELS"; Sibson 1981).  The weights depend only on geometry.

Definition used (area stealing): insert the query x into the parent set; its
Voronoi cell V+(x) takes area from the cells V(p) of its natural neighbours,
and w_p(x) = |V+(x) ∩ V(p)| / |V+(x)|.  A query that coincides with a parent
gets the Kronecker delta.

Parent set reading for partition factor s: parents sit on the lattice s Z^2
of signed beam indices, taken as an infinite lattice, so V(p) is the s x s
square centred on p.  The parents of a beam set are the lattice points that
receive a non-zero weight (> 1e-12) from at least one beam.  Because the
lattice is translation invariant, the weights of h depend only on (h mod s);
they are computed once per residue by exact half-plane polygon clipping.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

W_EPS = 1e-12


def clip_halfplane(poly, a, b, c):
    """Keep the part of polygon `poly` ([(x, y), ...]) with a*x + b*y <= c."""
    out = []
    n = len(poly)
    for i in range(n):
        p = poly[i]
        q = poly[(i + 1) % n]
        fp = a * p[0] + b * p[1] - c
        fq = a * q[0] + b * q[1] - c
        if fp <= 0:
            out.append(p)
        if (fp < 0 < fq) or (fq < 0 < fp):
            t = fp / (fp - fq)
            out.append((p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1])))
    return out


def area(poly) -> float:
    """Shoelace area of a simple polygon."""
    if len(poly) < 3:
        return 0.0
    s = 0.0
    for i in range(len(poly)):
        x0, y0 = poly[i]
        x1, y1 = poly[(i + 1) % len(poly)]
        s += x0 * y1 - x1 * y0
    return abs(s) * 0.5


def lattice_weights(x, s: int):
    """Sibson weights of query point x = (x0, x1) against the infinite lattice s Z^2.

    Returns {(p0, p1): w} with every weight > W_EPS (p in lattice units times s)."""
    x0, x1 = float(x[0]), float(x[1])
    c0 = int(np.floor(x0 / s))
    c1 = int(np.floor(x1 / s))
    if x0 == c0 * s and x1 == c1 * s:
        return {(c0 * s, c1 * s): 1.0}
    cand = [((c0 + i) * s, (c1 + j) * s) for i in (-1, 0, 1, 2) for j in (-1, 0, 1, 2)]
    # Voronoi cell of x among lattice ∪ {x}: intersection of the half-planes
    # |y - x|^2 <= |y - p|^2  <=>  2 (p - x) . y <= |p|^2 - |x|^2
    poly = [(x0 - s, x1 - s), (x0 + s, x1 - s), (x0 + s, x1 + s), (x0 - s, x1 + s)]
    for p in cand:
        a = 2.0 * (p[0] - x0)
        b = 2.0 * (p[1] - x1)
        c = p[0] ** 2 + p[1] ** 2 - x0 ** 2 - x1 ** 2
        poly = clip_halfplane(poly, a, b, c)
    total = area(poly)
    w = {}
    half = s / 2.0
    for p in cand:
        piece = poly
        piece = clip_halfplane(piece, 1.0, 0.0, p[0] + half)
        piece = clip_halfplane(piece, -1.0, 0.0, -(p[0] - half))
        piece = clip_halfplane(piece, 0.0, 1.0, p[1] + half)
        piece = clip_halfplane(piece, 0.0, -1.0, -(p[1] - half))
        ap = area(piece) / total
        if ap > W_EPS:
            w[p] = ap
    return w


def residue_table(s: int):
    """Weights for every residue (r0, r1) in [0, s)^2, as offsets from s*floor(h/s)."""
    table = {}
    for r0 in range(s):
        for r1 in range(s):
            w = lattice_weights((r0, r1), s)
            table[(r0, r1)] = [((p[0], p[1]), v) for p, v in sorted(w.items())]
    return table


class Partition:
    """Parents and the (sparse) weight matrix for one beam set and factor s."""

    def __init__(self, beams: np.ndarray, s: int):
        self.s = s
        self.beams = np.asarray(beams, dtype=np.int64)
        table = residue_table(s)
        rows, cols_h, vals = [], [], []
        for b, (hy, hx) in enumerate(self.beams):
            base = (s * (hy // s), s * (hx // s))
            for (o0, o1), v in table[(hy % s, hx % s)]:
                rows.append(b)
                cols_h.append((base[0] + o0, base[1] + o1))
                vals.append(v)
        parents = sorted(set(cols_h))
        self.parents = np.array(parents, dtype=np.int64).reshape(-1, 2)
        index = {p: i for i, p in enumerate(parents)}
        cols = [index[p] for p in cols_h]
        self.W = sp.csr_matrix((np.array(vals), (np.array(rows), np.array(cols))),
                               shape=(len(self.beams), len(parents)))

    @property
    def n_parents(self) -> int:
        return self.parents.shape[0]


# --------------------------------------------------------------------------
# Hex-ring parents and Sibson weights against a general parent set
# (section "Partitioned PRISM-EELS", parent selection and eq. nnw).
#
# Parent selection (Alg. 3 build step): the DC beam plus n_radial concentric
# rings; ring i (i = 0 .. n_radial-1) has radius (i + 1) / n_radial of the
# disc radius and n_angular (1 + i) samples at angles 2 pi k / (n_angular
# (1 + i)); each sample is snapped to the nearest beam of the set (ties to the
# smaller (h_y, h_x)) and duplicates are dropped.  The disc radius is given in
# beam-index units per axis (q = h / L: radius_y = qmax L_y, radius_x =
# qmax L_x).
#
# Weights: area stealing as above, with the parents a finite set.  The paper
# states no rule for beams outside the convex hull of the parents, where the
# Voronoi cell of the query is unbounded.  Reading used: a beam not strictly
# inside the hull takes the weights of its nearest point on the hull
# boundary, i.e. linear interpolation between the two ends of the nearest
# hull edge (the limit of the Sibson coordinates on that edge).
HULL_EPS = 1e-9


def hex_ring_parents(beams, n_radial, n_angular, radius_y, radius_x):
    """Parent beams [n, 2] (sorted by (h_y, h_x)) of a beam set on its disc."""
    beams = np.asarray(beams, dtype=np.int64)
    chosen = set()

    def snap(py, px):
        d2 = (beams[:, 0] - py) ** 2 + (beams[:, 1] - px) ** 2
        best = np.flatnonzero(d2 == d2.min())
        k = min(best, key=lambda i: (beams[i, 0], beams[i, 1]))
        return int(beams[k, 0]), int(beams[k, 1])

    chosen.add(snap(0.0, 0.0))
    for i in range(n_radial):
        frac = (i + 1) / n_radial
        m = n_angular * (1 + i)
        for k in range(m):
            t = 2.0 * np.pi * k / m
            chosen.add(snap(frac * radius_y * np.sin(t), frac * radius_x * np.cos(t)))
    return np.array(sorted(chosen), dtype=np.int64).reshape(-1, 2)


def convex_hull(points):
    """Counter-clockwise hull vertices (no collinear points), monotone chain."""
    pts = sorted(set(map(tuple, np.asarray(points, dtype=float))))
    if len(pts) < 3:
        return pts

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    return lower[:-1] + upper[:-1]


def _hull_projection(x, hull):
    """(inside strictly?, {vertex: weight}) for the hull rule."""
    n = len(hull)
    inside = True
    best = None
    for i in range(n):
        a = np.array(hull[i])
        b = np.array(hull[(i + 1) % n])
        e = b - a
        # signed distance of x to the edge's line (positive inside for CCW order)
        s = (e[0] * (x[1] - a[1]) - e[1] * (x[0] - a[0])) / np.hypot(e[0], e[1])
        if s <= HULL_EPS:
            inside = False
        t = float(np.clip(np.dot(x - a, e) / np.dot(e, e), 0.0, 1.0))
        d = np.hypot(*(a + t * e - x))
        if best is None or d < best[0]:
            best = (d, tuple(hull[i]), tuple(hull[(i + 1) % n]), t)
    _, a, b, t = best
    w = {}
    for p, v in ((a, 1.0 - t), (b, t)):
        if v > W_EPS:
            w[(int(round(p[0])), int(round(p[1])))] = w.get((int(round(p[0])), int(round(p[1]))), 0.0) + v
    return inside, w


def general_weights(x, parents, hull=None):
    """Sibson weights {(p0, p1): w} of query x against the finite parent set
    `parents` [n, 2], with the hull rule for queries not strictly inside."""
    x = np.asarray(x, dtype=float)
    P = [tuple(map(float, p)) for p in np.asarray(parents)]
    for p in P:
        if p[0] == x[0] and p[1] == x[1]:
            return {(int(p[0]), int(p[1])): 1.0}
    hull = convex_hull(parents) if hull is None else hull
    inside, w = _hull_projection(x, hull)
    if not inside:
        return w
    # Voronoi cell of x among the parents and x.  It is bounded (x is strictly
    # inside the hull) but may reach far out when x is near the hull: start
    # from a box around x and enlarge it until no vertex of the cell lies on it.
    span = max(max(abs(p[0] - x[0]), abs(p[1] - x[1])) for p in P)
    while True:
        cell = [(x[0] - span, x[1] - span), (x[0] + span, x[1] - span),
                (x[0] + span, x[1] + span), (x[0] - span, x[1] + span)]
        for p in P:
            cell = clip_halfplane(cell, 2.0 * (p[0] - x[0]), 2.0 * (p[1] - x[1]),
                                  p[0] ** 2 + p[1] ** 2 - x[0] ** 2 - x[1] ** 2)
        reach = max(max(abs(v[0] - x[0]), abs(v[1] - x[1])) for v in cell)
        if reach < span * (1.0 - 1e-9):
            break
        span *= 8.0
    total = area(cell)
    out = {}
    for p in P:
        # natural neighbours only: the cell reaches p's bisector with x
        line = [2.0 * (p[0] - x[0]) * v[0] + 2.0 * (p[1] - x[1]) * v[1] -
                (p[0] ** 2 + p[1] ** 2 - x[0] ** 2 - x[1] ** 2) for v in cell]
        if max(line) < -1e-9 * (1.0 + span * span):
            continue
        piece = cell
        for q in P:
            if q == p:
                continue
            piece = clip_halfplane(piece, 2.0 * (q[0] - p[0]), 2.0 * (q[1] - p[1]),
                                   q[0] ** 2 + q[1] ** 2 - p[0] ** 2 - p[1] ** 2)
            if len(piece) < 3:
                break
        a = area(piece) / total
        if a > W_EPS:
            out[(int(p[0]), int(p[1]))] = a
    return out


class HexPartition:
    """Hex-ring parents and their (sparse) weight matrix for one beam set;
    same interface as Partition."""

    def __init__(self, beams, n_radial, n_angular, radius_y, radius_x):
        self.beams = np.asarray(beams, dtype=np.int64)
        self.parents = hex_ring_parents(self.beams, n_radial, n_angular, radius_y, radius_x)
        index = {tuple(p): i for i, p in enumerate(self.parents.tolist())}
        hull = convex_hull(self.parents)
        rows, cols, vals = [], [], []
        for b, h in enumerate(self.beams):
            for p, v in sorted(general_weights(h, self.parents, hull).items()):
                rows.append(b)
                cols.append(index[p])
                vals.append(v)
        self.W = sp.csr_matrix((np.array(vals), (np.array(rows), np.array(cols))),
                               shape=(len(self.beams), len(self.parents)))

    @property
    def n_parents(self) -> int:
        return self.parents.shape[0]
