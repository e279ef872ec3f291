"""Seeded unstructured triangulations around the lamina.

The paper's body-fitted grid is an unstructured triangulation of a thin band
around the body (Sec. Hybrid lattice Boltzmann method). This module places
nodes and triangulates them; it holds none of the method's arithmetic (no
control volumes, stencils or interpolation), so both the GPU library and the
CPU oracle can take the same mesh from it.

A mesh covers the rectangle [-W/2, W/2] x [-H/2, H/2] (the local frame, the
lamina centre at the origin) minus the lamina [-b/2, b/2] x [-T/2, T/2]. Its
nodes are spaced h_wall on the lamina's surface, growing with the distance d
from it as min(h_far, h_wall + grading d) inside, and h_far on the outer
boundary. Node types follow the library and the oracle: 0 interior
(discretization), 1 interface (outer boundary: interpolation node), 2 wall.
"""
from __future__ import annotations

import math

import numpy as np

INTERIOR, INTERFACE, WALL = 0, 1, 2


def _perimeter(x0, x1, y0, y1, spacing_x, spacing_y):
    """Points along the rectangle's boundary, counter-clockwise from (x0,
    y0), each side cut into equal segments no longer than the spacing."""
    nx = max(1, math.ceil((x1 - x0) / spacing_x - 1e-9))
    ny = max(1, math.ceil((y1 - y0) / spacing_y - 1e-9))
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)
    pts = [(x, y0) for x in xs[:-1]] + [(x1, y) for y in ys[:-1]] + \
          [(x, y1) for x in xs[:0:-1]] + [(x0, y) for y in ys[:0:-1]]
    return np.array(pts, dtype=float)


def _dist_rect(p, hx, hy):
    """Distance from points p to the rectangle |x| <= hx, |y| <= hy (0 inside)."""
    dx = np.maximum(np.abs(p[:, 0]) - hx, 0.0)
    dy = np.maximum(np.abs(p[:, 1]) - hy, 0.0)
    return np.hypot(dx, dy)


def lamina_triangulation(W, H, b=0.0, T=1.0, h_wall=0.5, h_far=1.0, grading=0.3, seed=0, smooth=0):
    """Unstructured triangulation around the lamina (see the module header).

    Returns ``(xy, node_type, tri)``: coordinates [n, 2] (float64), types [n]
    (int32) and counter-clockwise triangles [m, 3] (int32). Interior nodes
    come from seeded dart throwing with the graded spacing, so no two meshes
    of different seeds share a structure; the triangulation is Delaunay,
    with the triangles inside the lamina removed. Raises ValueError when the
    result does not cover the region exactly (then change the spacing or the
    seed)."""
    from scipy.spatial import Delaunay, cKDTree

    if not (W > 0 and H > 0 and h_wall > 0 and h_far >= h_wall):
        raise ValueError("need W, H > 0 and h_far >= h_wall > 0")
    body = b > 0.0
    hb, ht = 0.5 * b, 0.5 * T
    if body and not (hb + h_far < 0.5 * W and ht + h_far < 0.5 * H):
        raise ValueError("the lamina must lie inside the rectangle with a margin")
    rng = np.random.default_rng(seed)

    outer = _perimeter(-0.5 * W, 0.5 * W, -0.5 * H, 0.5 * H, h_far, h_far)
    wall = _perimeter(-hb, hb, -ht, ht, h_wall, h_wall) if body else np.zeros((0, 2))

    def spacing(p):
        d = _dist_rect(p, hb, ht) if body else np.full(len(p), np.inf)
        return np.minimum(h_far, h_wall + grading * d)

    # dart throwing: candidates in random order, accepted when no accepted
    # node (boundary nodes first) lies closer than 0.8 of the local spacing
    # and the boundaries are at least half of it away
    area = W * H
    ncand = int(4.0 * area / (h_wall * h_far)) + 64
    cand = np.column_stack([rng.uniform(-0.5 * W, 0.5 * W, ncand), rng.uniform(-0.5 * H, 0.5 * H, ncand)])
    hc = spacing(cand)
    margin_out = np.minimum(0.5 * W - np.abs(cand[:, 0]), 0.5 * H - np.abs(cand[:, 1]))
    keep = margin_out >= 0.5 * hc
    if body:
        keep &= _dist_rect(cand, hb, ht) >= 0.5 * hc
    cand, hc = cand[keep], hc[keep]
    # in chunks: a candidate is checked against the nodes accepted before its
    # chunk with a k-d tree, then against the earlier ones of its own chunk
    pts = np.vstack([outer, wall])
    chunk = 4096
    for c0 in range(0, len(cand), chunk):
        c, h = cand[c0:c0 + chunk], hc[c0:c0 + chunk]
        d, _ = cKDTree(pts).query(c, k=1)
        ok = np.nonzero(d >= 0.8 * h)[0]
        if len(ok) == 0:
            continue
        sub, subh = c[ok], h[ok]
        earlier = [[] for _ in range(len(sub))]
        for i, j in cKDTree(sub).query_pairs(0.8 * subh.max()):
            earlier[max(i, j)].append(min(i, j))
        taken = np.zeros(len(sub), bool)
        for j in range(len(sub)):
            r2 = (0.8 * subh[j]) ** 2
            taken[j] = not any(taken[i] and ((sub[i] - sub[j]) ** 2).sum() < r2 for i in earlier[j])
        pts = np.vstack([pts, sub[taken]])
    xy = np.asarray(pts, dtype=float)
    n_out, n_wall = len(outer), len(wall)
    node_type = np.full(len(xy), INTERIOR, np.int32)
    node_type[:n_out] = INTERFACE
    node_type[n_out:n_out + n_wall] = WALL
    # number the nodes along a Z-order curve of unit cells, so that nodes
    # with nearby numbers are near each other (and share neighbours)
    cell = np.floor((xy - xy.min(axis=0)) / h_far).astype(np.int64)
    key = np.zeros(len(xy), np.int64)
    for bit in range(20):
        key |= ((cell[:, 0] >> bit) & 1) << (2 * bit) | ((cell[:, 1] >> bit) & 1) << (2 * bit + 1)
    order = np.lexsort((xy[:, 1], xy[:, 0], key))
    xy, node_type = xy[order], node_type[order]

    def triangulate(xy):
        dl = Delaunay(xy)
        if len(getattr(dl, "coplanar", [])):
            raise ValueError("points left out of the triangulation")
        tri = dl.simplices.astype(np.int64)
        if body:
            cen = xy[tri].mean(axis=1)
            tri = tri[~((np.abs(cen[:, 0]) < hb) & (np.abs(cen[:, 1]) < ht))]
        return tri
    tri = triangulate(xy)
    # optional Laplacian smoothing: each interior node moves to the mean of
    # its neighbours, then the nodes are triangulated again
    inner = node_type == INTERIOR
    for _ in range(smooth):
        e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
        e = np.concatenate([e, e[:, ::-1]])
        acc = np.zeros_like(xy)
        np.add.at(acc, e[:, 0], xy[e[:, 1]])
        deg = np.bincount(e[:, 0], minlength=len(xy)).astype(float)
        mean = acc / np.maximum(deg, 1.0)[:, None]
        xy = np.where(inner[:, None], mean, xy)
        tri = triangulate(xy)
    # counter-clockwise
    a = xy[tri]
    cross = (a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1]) - \
            (a[:, 2, 0] - a[:, 0, 0]) * (a[:, 1, 1] - a[:, 0, 1])
    flip = cross < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    cross = np.abs(cross)
    if not np.all(cross > 1e-12 * h_wall * h_wall):
        raise ValueError("degenerate triangle")
    _check_cover(xy, node_type, tri, W, H, hb, ht, body, 0.5 * cross.sum())
    return xy, node_type, tri.astype(np.int32)


def _check_cover(xy, node_type, tri, W, H, hb, ht, body, area):
    """The mesh covers the rectangle minus the lamina: the areas agree and
    every edge with one triangle lies on the outer boundary (both ends
    interface nodes) or on the lamina (both ends wall nodes); every node is
    used."""
    want = W * H - (4 * hb * ht if body else 0.0)
    if abs(area - want) > 1e-9 * want:
        raise ValueError(f"mesh area {area} differs from the region's {want}")
    e = np.sort(np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]]), axis=1)
    uniq, cnt = np.unique(e, axis=0, return_counts=True)
    if np.any(cnt > 2):
        raise ValueError("an edge shared by more than two triangles")
    bnd = uniq[cnt == 1]
    t0, t1 = node_type[bnd[:, 0]], node_type[bnd[:, 1]]
    if not np.all(t0 == t1) or np.any(t0 == INTERIOR):
        raise ValueError("a boundary edge leaves the outer boundary or the lamina")
    p, q = xy[bnd[:, 0]], xy[bnd[:, 1]]
    on_side = (np.isclose(p[:, 0], q[:, 0]) & np.isclose(np.abs(p[:, 0]), np.where(t0 == WALL, hb, 0.5 * W))) | \
              (np.isclose(p[:, 1], q[:, 1]) & np.isclose(np.abs(p[:, 1]), np.where(t0 == WALL, ht, 0.5 * H)))
    if not np.all(on_side):
        raise ValueError("a boundary edge cuts a corner")
    if len(np.unique(tri)) != len(xy):
        raise ValueError("a node belongs to no triangle")
