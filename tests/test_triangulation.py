"""The host triangulation of the prior construction (lf_triangulate, no
device work): Delaunay by its definition (no point strictly inside any
triangle's circumcircle, checked with exact integers), a triangulation of
the convex hull (Euler's count and the hull's area), and scipy's Delaunay
where the points are in general position (the triangulation is unique)."""
import numpy as np
import pytest

import paper_2003_11076_amd as LF


def _incircle(a, b, c, d):
    adx, ady, bdx, bdy, cdx, cdy = a[0] - d[0], a[1] - d[1], b[0] - d[0], b[1] - d[1], c[0] - d[0], c[1] - d[1]
    return ((adx * adx + ady * ady) * (bdx * cdy - bdy * cdx) - (bdx * bdx + bdy * bdy) * (adx * cdy - ady * cdx)
            + (cdx * cdx + cdy * cdy) * (adx * bdy - ady * bdx))


def _hull(pts):
    """Monotone chain; returns (vertices, number of points on the boundary, twice the area)."""
    P = sorted(set(map(tuple, pts)))
    if len(P) < 3:
        return P, len(P), 0

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])
    lo, up = [], []
    for p in P:
        while len(lo) >= 2 and cross(lo[-2], lo[-1], p) <= 0:
            lo.pop()
        lo.append(p)
    for p in reversed(P):
        while len(up) >= 2 and cross(up[-2], up[-1], p) <= 0:
            up.pop()
        up.append(p)
    H = lo[:-1] + up[:-1]
    area2 = sum(H[i][0] * H[(i + 1) % len(H)][1] - H[(i + 1) % len(H)][0] * H[i][1] for i in range(len(H)))
    on = 0
    for p in P:
        for i in range(len(H)):
            a, b = H[i], H[(i + 1) % len(H)]
            if cross(a, b, p) == 0 and min(a[0], b[0]) <= p[0] <= max(a[0], b[0]) and \
                    min(a[1], b[1]) <= p[1] <= max(a[1], b[1]):
                on += 1
                break
    return H, on, area2


def _check_delaunay(pts, tris):
    pts = [tuple(map(int, p)) for p in pts]
    n = len(set(pts))
    _, h, area2 = _hull(pts)
    assert len(tris) == 2 * n - h - 2                      # a triangulation of all points
    tot = 0
    for t in tris:
        a, b, c = (pts[i] for i in t)
        o = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
        assert o > 0                                       # counter-clockwise, not degenerate
        tot += o
    assert tot == area2                                    # covers the hull exactly
    for t in tris:
        a, b, c = (pts[i] for i in t)
        for d in pts:
            assert _incircle(a, b, c, d) <= 0              # empty circumcircle


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_points_match_scipy(seed):
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    xy = np.unique(rng.integers(0, 2000, size=(300, 2)), axis=0).astype(np.int32)
    rng.shuffle(xy)
    tris = LF.lf_triangulate(xy)
    ours = {tuple(sorted(t)) for t in tris.tolist()}
    ref = {tuple(sorted(t)) for t in Delaunay(xy.astype(float)).simplices.tolist()}
    # general position with probability ~1: the Delaunay triangulation is unique
    assert ours == ref
    _check_delaunay(xy, tris)


def test_grid_points_with_corners_and_collinear_rows():
    xs, ys = np.arange(2, 80, 5), np.arange(2, 50, 5)
    xy = [(x, y) for y in ys for x in xs] + [(0, 0), (79, 0), (0, 49), (79, 49), (0, 17), (40, 49)]
    xy = np.array(xy, np.int32)
    tris = LF.lf_triangulate(xy)
    _check_delaunay(xy, tris)


def test_degenerate_inputs():
    assert len(LF.lf_triangulate(np.zeros((0, 2), np.int32))) == 0
    assert len(LF.lf_triangulate(np.array([[1, 1], [5, 5], [9, 9], [13, 13]], np.int32))) == 0   # collinear
    tris = LF.lf_triangulate(np.array([[0, 0], [10, 0], [0, 10], [10, 0]], np.int32))           # a duplicate
    assert len(tris) == 1
    with pytest.raises(LF.LFError):
        LF.lf_triangulate(np.array([[0, 0], [20000, 1], [3, 3]], np.int32))
