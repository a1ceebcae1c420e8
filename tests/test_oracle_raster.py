"""Pins for the oracle rasteriser (light-view shadow map and camera key buffer).

The shadow-map pass is the vanilla rasterised depth map the method takes as
input (paper Sec. 1 and 3.1).  The rasteriser is pinned against
(i) watertightness of a triangulated rectangle (every texel centre inside is
covered exactly once), (ii) the closed-form texel set of a snapped
rectangle, (iii) the analytic affine depth of a plane, (iv) an exact
rational brute force on tiny random scenes, and (v) the clip-space drop rule.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from nsm_synth import SplitMix64

W = H = 64
# world -> clip = identity with w = 1: ndc equals world coordinates.
IDENT = np.eye(4, dtype=np.float32)


def to_ndc(X, n):
    """Fixed-point screen coordinate X (1/256 px) -> float32 ndc, exact."""
    return np.float32(X / (128.0 * n) - 1.0)


def tri_from_fixed(pts, zs):
    return np.array([[to_ndc(x, W), to_ndc(y, H), z] for (x, y), z in zip(pts, zs)], np.float32)


def rect_tris(x0, y0, x1, y1, z=0.5):
    a, b, c, d = (x0, y0), (x1, y0), (x1, y1), (x0, y1)
    return np.stack([tri_from_fixed([a, b, c], [z] * 3), tri_from_fixed([a, c, d], [z] * 3)])


def rect_closed_form(x0, y0, x1, y1):
    """Texels whose centre (256i+128, 256j+128) lies in (x0, x1] x (y0, y1]:
    left and bottom edges exclusive, right and top edges inclusive (the tie
    rule for counter-clockwise triangles with y growing upward)."""
    out = np.zeros((H, W), np.uint32)
    for j in range(H):
        for i in range(W):
            cx, cy = 256 * i + 128, 256 * j + 128
            out[j, i] = 1 if (x0 < cx <= x1 and y0 < cy <= y1) else 0
    return out


@pytest.mark.parametrize("rect", [(0, 0, 256 * 64, 256 * 64), (300, 1000, 9000, 12000),
                                  (128, 128, 128 + 256 * 10, 128 + 256 * 7), (-5000, 700, 4000, 30000)])
def test_rectangle_closed_form(rect):
    counts, stats = oracle.raster(rect_tris(*rect), IDENT, W, H, "count")
    assert stats[0] == 0
    np.testing.assert_array_equal(counts, rect_closed_form(*rect))


def test_watertight_jittered_grid():
    """A rectangle split into a grid of jittered quads, each into two triangles
    along a random diagonal: every texel covered exactly once inside."""
    rng = SplitMix64(7)
    x0, y0, x1, y1 = 700, 900, 15000, 15500
    n = 9
    gx = np.linspace(x0, x1, n + 1).round().astype(np.int64)
    gy = np.linspace(y0, y1, n + 1).round().astype(np.int64)
    P = np.zeros((n + 1, n + 1, 2), np.int64)
    for a in range(n + 1):
        for b in range(n + 1):
            jx = 0 if a in (0, n) else int(rng.uniform(-300, 300))
            jy = 0 if b in (0, n) else int(rng.uniform(-300, 300))
            P[a, b] = (gx[a] + jx, gy[b] + jy)
    tris = []
    for a in range(n):
        for b in range(n):
            p00, p10, p11, p01 = P[a, b], P[a + 1, b], P[a + 1, b + 1], P[a, b + 1]
            if rng.uniform() < 0.5:
                tris += [[p00, p10, p11], [p00, p11, p01]]
            else:
                tris += [[p00, p10, p01], [p10, p11, p01]]
            # random winding: the rasteriser must not cull
            if rng.uniform() < 0.5:
                tris[-1] = [tris[-1][0], tris[-1][2], tris[-1][1]]
    soup = np.stack([tri_from_fixed([tuple(v) for v in t], [0.25] * 3) for t in tris])
    counts, stats = oracle.raster(soup, IDENT, W, H, "count")
    np.testing.assert_array_equal(counts, rect_closed_form(x0, y0, x1, y1))
    assert stats == (0, 0, 0)


def test_plane_depth_is_affine():
    """Depth of a planar triangle equals the plane's affine value at the texel
    centre (computed exactly with rationals) to within one float32 ulp."""
    pts = [(1000, 800), (15000, 3000), (5000, 15800)]
    zs = [np.float32(0.1), np.float32(0.7), np.float32(0.35)]
    tri = tri_from_fixed(pts, zs)[None]
    depth, _ = oracle.raster(tri, IDENT, W, H, "depth")
    covered = depth != oracle.EMPTY_DEPTH
    assert covered.sum() > 500
    # plane through the three (X, Y, z) points, exact
    (xa, ya), (xb, yb), (xc, yc) = pts
    za, zb, zc = (Fraction(float(z)) for z in zs)
    det = Fraction((xb - xa) * (yc - ya) - (yb - ya) * (xc - xa))
    for j, i in zip(*np.nonzero(covered)):
        px, py = 256 * i + 128, 256 * j + 128
        # barycentric weights by Cramer's rule
        l1 = Fraction((px - xa) * (yc - ya) - (py - ya) * (xc - xa)) / det
        l2 = Fraction((xb - xa) * (py - ya) - (yb - ya) * (px - xa)) / det
        z = za + l1 * (zb - za) + l2 * (zc - za)
        got = np.array([depth[j, i]], np.uint32).view(np.float32)[0]
        want = np.float32(float(z))
        assert abs(int(np.array([got]).view(np.int32)[0]) - int(np.array([want]).view(np.int32)[0])) <= 1


def _brute_force(tris, w, h):
    """Exact rational reference: snap vertices the way the specification
    does (round-half-even of 256 * screen coordinate), test coverage with
    exact orientation signs, interpolate depth exactly, keep the nearest."""
    best = {}
    for t, tri in enumerate(tris):
        X, Y, Z = [], [], []
        for v in tri:
            sx = (np.float32(v[0]) * np.float32(0.5) + np.float32(0.5)) * np.float32(w)
            sy = (np.float32(v[1]) * np.float32(0.5) + np.float32(0.5)) * np.float32(h)
            X.append(int(np.rint(np.float32(sx * np.float32(256.0)))))
            Y.append(int(np.rint(np.float32(sy * np.float32(256.0)))))
            Z.append(Fraction(float(v[2])))
        area = (X[1] - X[0]) * (Y[2] - Y[0]) - (Y[1] - Y[0]) * (X[2] - X[0])
        if area == 0:
            continue
        if area < 0:
            X[1], X[2], Y[1], Y[2], Z[1], Z[2] = X[2], X[1], Y[2], Y[1], Z[2], Z[1]
            area = -area
        edges = [(1, 2), (2, 0), (0, 1)]
        for j in range(h):
            for i in range(w):
                px, py = 256 * i + 128, 256 * j + 128
                ok, lam = True, []
                for (a, b) in edges:
                    e = (X[b] - X[a]) * (py - Y[a]) - (Y[b] - Y[a]) * (px - X[a])
                    dx, dy = X[b] - X[a], Y[b] - Y[a]
                    top_left = dy > 0 or (dy == 0 and dx < 0)
                    if not (e > 0 or (e == 0 and top_left)):
                        ok = False
                        break
                    lam.append(e)
                if not ok:
                    continue
                z = sum(Fraction(l) * zz for l, zz in zip(lam, Z)) / area
                if 0 <= z <= 1:
                    zf = np.float32(float(z))
                    key = (float(zf), t)
                    if (j, i) not in best or key < best[(j, i)]:
                        best[(j, i)] = key
    return best


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_zbuffer_matches_exact_brute_force(seed):
    """Random overlapping triangles on a 16x16 target: same covered texels,
    same winning triangle, depth within one ulp of the exact value."""
    w = h = 16
    rng = SplitMix64(100 + seed)
    tris = np.zeros((12, 3, 3), np.float32)
    for t in range(12):
        for v in range(3):
            tris[t, v] = [rng.uniform(-1.2, 1.2), rng.uniform(-1.2, 1.2), rng.uniform(0.0, 1.0)]
    # a shared edge between triangles 0 and 1 exercises the tie rule
    tris[1, 0], tris[1, 1] = tris[0, 1], tris[0, 0]
    keys, _ = oracle.raster(tris, IDENT, w, h, "key")
    depth, _ = oracle.raster(tris, IDENT, w, h, "depth")
    best = _brute_force(tris, w, h)
    for j in range(h):
        for i in range(w):
            k = int(keys[j, i])
            if (j, i) not in best:
                assert k == oracle.EMPTY_KEY and depth[j, i] == oracle.EMPTY_DEPTH
                continue
            zb, tb = best[(j, i)]
            got_t = k & 0xFFFFFFFF
            got_z = np.array([k >> 32], np.uint32).view(np.float32)[0]
            assert (k >> 32) == int(depth[j, i])
            ulp = abs(int(np.array([got_z], np.float32).view(np.int32)[0])
                      - int(np.array([zb], np.float32).view(np.int32)[0]))
            assert ulp <= 1
            if ulp == 0:
                assert got_t == tb


def test_behind_camera_dropped():
    tri = np.array([[[0, 0, 0.5], [0.5, 0, 0.5], [0, 0.5, 0.5]]], np.float32)
    m = IDENT.copy()
    m[3] = [0, 0, 0, -1]          # w = -1 for every vertex
    depth, stats = oracle.raster(tri, m, W, H, "depth")
    assert stats[0] == 1 and (depth == oracle.EMPTY_DEPTH).all()


def test_camera_key_lowest_id_wins_ties():
    t = rect_tris(0, 0, 256 * 64, 256 * 64, z=0.5)
    tris = np.concatenate([t, t])            # ids 2,3 duplicate 0,1
    keys, _ = oracle.raster(tris, IDENT, W, H, "key")
    ids = keys & np.uint64(0xFFFFFFFF)
    assert set(np.unique(ids).tolist()) <= {0, 1}
