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
