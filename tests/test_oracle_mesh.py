"""Pins of the oracle's body-fitted grid and its finite-volume matrices
S_ik and C_ik (Eq.(ulbe), Sec. 3).

The paper cites S_ik and C_ik without giving them; the oracle takes the
median-dual control volume with piecewise-linear f. These tests check that
assembly against closed forms computed here independently:

* streaming: by the divergence theorem the outflow through the boundary of a
  control volume equals the integral of c.grad f over it, and each triangle
  gives one third of its area to each vertex, so
  S_ik = -(1/V_P) sum_{T ni P} (|T|/3) c_i . grad(phi_k on T);
* collision: the integral of a vertex's own shape function over its part of
  a triangle is 11/54 |T|, that of either other vertex 7/108 |T|;
* consistency: sum_k C_ik = 1, sum_k S_ik = 0, and the scheme is exact on
  linear fields, sum_k S_ik (a . x_k) = -c_i . a.
"""
import numpy as np
import pytest

from paper_2006_13631_amd.workloads import graded_nodes

# graded lamina grids (spacing growing away from the lamina)
GX = graded_nodes(15, 0.5, 1.4, 2.0, fine=2.0)
GY = graded_nodes(10, 0.5, 1.5, 2.0)

MESHES = [
    ("graded", dict(X=GX, Y=GY, b=3.0)),
    ("graded", dict(X=graded_nodes(11, 1.0, 1.3, 3.0), Y=graded_nodes(8, 1.0, 1.3, 3.0), b=0.0)),
    ("lamina", dict(nux=12, nuy=8, h=1.0, b=4.0)),
    ("lamina", dict(nux=13, nuy=10, h=0.5, b=3.0)),
    ("lamina", dict(nux=9, nuy=6, h=1.0, b=0.0)),
    ("periodic", dict(nx=6, ny=5, h=1.0)),
    ("channel", dict(nx=5, ny=6, h=0.7)),
]


def _mesh(oracle, kind, kw):
    if kind == "graded":
        return oracle.Mesh.lamina_coords(kw["X"], kw["Y"], kw["b"])
    if kind == "lamina":
        return oracle.Mesh.lamina(kw["nux"], kw["nuy"], kw["h"], kw["b"])
    if kind == "periodic":
        return oracle.Mesh.periodic(kw["nx"], kw["ny"], kw["h"])
    return oracle.Mesh.channel(kw["nx"], kw["ny"], kw["h"])


def _dense(nbr, M):
    """[nnode][k] (or [nnode][9][k]) neighbour-slot matrix -> dense [9][N][N]"""
    N = nbr.shape[0]
    if M.ndim == 2:
        D = np.zeros((N, N))
        for p in range(N):
            for k, q in enumerate(nbr[p]):
                if q >= 0:
                    D[p, q] += M[p, k]
        return D
    D = np.zeros((9, N, N))
    for p in range(N):
        for k, q in enumerate(nbr[p]):
            if q >= 0:
                D[:, p, q] += M[p, :, k]
    return D


def _closed_forms(oracle, m):
    cx, cy, _ = oracle.d2q9()
    tri, txy = m.triangles()
    N = m.nnode
    V = np.zeros(N)
    S = np.zeros((9, N, N))
    Cm = np.zeros((N, N))
    for t in range(m.ntri):
        P = txy[t]
        area = 0.5 * ((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]))
        assert area > 0
        # gradients of the linear shape functions: grad phi_a = perp(opposite edge) / (2 area)
        grads = []
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            ex, ey = P[c] - P[b]
            grads.append(np.array([-ey, ex]) / (2 * area))
        for a in range(3):
            p = tri[t, a]
            V[p] += area / 3
            for j in range(3):
                q = tri[t, j]
                S[:, p, q] -= (area / 3) * (cx * grads[j][0] + cy * grads[j][1])
                Cm[p, q] += area * (11.0 / 54.0 if j == a else 7.0 / 108.0)
    return V, S / V[None, :, None], Cm / V[:, None]


@pytest.mark.parametrize("kind,kw", MESHES)
def test_stencil_matches_closed_forms(oracle, kind, kw):
    m = _mesh(oracle, kind, kw)
    nbr, S, Cm, V = m.stencil()
    V0, S0, C0 = _closed_forms(oracle, m)
    assert np.max(np.abs(V - V0)) < 1e-13
    Sd = _dense(nbr, S)
    Cd = _dense(nbr, Cm)
    assert np.max(np.abs(Sd - S0)) < 1e-13
    assert np.max(np.abs(Cd - C0)) < 1e-14


@pytest.mark.parametrize("kind,kw", MESHES)
def test_stencil_consistency(oracle, kind, kw):
    m = _mesh(oracle, kind, kw)
    nbr, S, Cm, V = m.stencil()
    cx, cy, _ = oracle.d2q9()
    x, y, _ = m.nodes()
    assert np.all(nbr[:, 0] == np.arange(m.nnode))  # k = 0 is the pivotal node
    assert np.max(np.abs(Cm.sum(1) - 1.0)) < 1e-14
    assert np.max(np.abs(S.sum(2))) < 1e-13
    # linear fields along a periodic direction are not single-valued
    dirs = {"lamina": ((1.0, 0.0), (0.0, 1.0), (0.3, -0.7)), "graded": ((1.0, 0.0), (0.0, 1.0), (0.3, -0.7)),
            "channel": ((0.0, 1.0),), "periodic": ()}
    for a in dirs[kind]:
        lin = a[0] * x + a[1] * y
        got = np.einsum("pik,pk->pi", S, np.where(nbr >= 0, lin[nbr], 0.0))
        want = -(cx * a[0] + cy * a[1])[None, :]
        assert np.max(np.abs(got - want)) < 1e-12


def test_grid_geometry(oracle):
    """Lamina grid: 2(b/h + 1) wall nodes, the outer ring are interface nodes,
    the meshed area is the grid rectangle minus the lamina slot."""
    nux, nuy, h, b = 16, 10, 1.0, 6.0
    m = oracle.Mesh.lamina(nux, nuy, h, b)
    x, y, t = m.nodes()
    assert (t == oracle.NODE_WALL).sum() == 2 * (int(b / h) + 1)
    assert (t == oracle.NODE_INTERFACE).sum() == 2 * (nux + nuy) - 4
    wall = t == oracle.NODE_WALL
    assert np.allclose(np.abs(y[wall]), 0.5 * h) and np.all(np.abs(x[wall]) <= b / 2 + 1e-12)
    _, _, _, V = m.stencil()
    area = (nux - 1) * (nuy - 1) * h * h - b * h
    assert abs(V.sum() - area) < 1e-12
    # mirror-symmetric diagonals: the triangle set maps onto itself under x -> -x
    m2 = oracle.Mesh.lamina(nux + 1, nuy, h, b)
    _, txy = m2.triangles()
    key = lambda P: tuple(sorted((round(a, 9), round(c, 9)) for a, c in P))
    fwd = {key(P) for P in txy}
    mir = {key(np.c_[-P[:, 0], P[:, 1]]) for P in txy}
    assert fwd == mir


@pytest.mark.parametrize("graded", [False, True])
def test_point_location_vs_exhaustive(oracle, graded):
    m = oracle.Mesh.lamina_coords(GX, GY, 3.0) if graded else oracle.Mesh.lamina(10, 8, 1.0, 4.0)
    tri, txy = m.triangles()
    rng = np.random.default_rng(7)
    pts = rng.uniform([-6, -4.5], [5, 4.5], size=(400, 2))
    # add points on edges and vertices
    pts = np.vstack([pts, txy.reshape(-1, 2)[:60], 0.5 * (txy[:40, 0] + txy[:40, 1])])
    for px, py in pts:
        t, lam = m.locate(px, py)
        inside = []
        for u in range(m.ntri):
            P = txy[u]
            T = np.array([[P[1, 0] - P[0, 0], P[2, 0] - P[0, 0]], [P[1, 1] - P[0, 1], P[2, 1] - P[0, 1]]])
            l12 = np.linalg.solve(T, [px - P[0, 0], py - P[0, 1]])
            l = np.array([1 - l12.sum(), l12[0], l12[1]])
            if np.all(l >= -1e-12):
                inside.append((u, l))
        if not inside:
            assert t == -1
        else:
            assert t == inside[0][0]
            assert np.allclose(lam, inside[0][1], atol=1e-12)
            assert np.allclose(lam @ txy[t], [px, py], atol=1e-12)
