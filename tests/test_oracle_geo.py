"""Pins of the geometry oracle: DSM interpolation, ray / DSM intersection,
footprints, footprint overlaps and the Eq. (3) patch transfer (Sec. 3.1).

Independent checks: node values and planes that bilinear interpolation
reproduces exactly (dyadic values, exact in float32); closed-form
intersections with flat and tilted planes; a brute-force walk along the ray
for the first crossing over hills; the scene generator's own projection for
round trips; closed-form overlap areas (rectangles, a square and its 45
degree turn, containment, disjoint) and a dense point-in-polygon count;
Eq. (3) with k = 0 and with a pure translation over flat ground."""
import math

import numpy as np
import pytest

from oracle import geo as G
from synth import aerial as A
from synth import geo as SG

F, CX, CY, W, H = A.F_PX, A.CX, A.CY, A.IMG_W, A.IMG_H


def flat(h0=20.0):
    return SG.plane_dsm(40, 40, -240.0, -240.0, 12.0, 0.0, 0.0, h0)


def tilted():
    return SG.plane_dsm(64, 64, -256.0, -256.0, 8.0, 0.125, -0.0625, 20.0)   # dyadic: exact in float32


def hills():
    return SG.make_geo_flight(21, n_strips=2, imgs_per_strip=6)


def test_heights_at_nodes_and_clamped():
    g = hills()
    d = g["dsm"]
    for i, j in [(0, 0), (3, 7), (d["nx"] - 1, d["ny"] - 1), (d["nx"] - 1, 0)]:
        x, y = d["x0"] + i * d["cell"], d["y0"] + j * d["cell"]
        assert G.dsm_height(d, x, y) == float(d["h"][j, i])
    assert G.dsm_height(d, d["x0"] - 500.0, d["y0"] - 500.0) == float(d["h"][0, 0])


def test_bilinear_reproduces_plane():
    d = tilted()
    rng = np.random.default_rng(1)
    for x, y in rng.uniform(-250.0, 250.0, (50, 2)):
        assert abs(G.dsm_height(d, x, y) - (0.125 * x - 0.0625 * y + 20.0)) < 1e-12


@pytest.mark.parametrize("u,v", [(0.0, 0.0), (W, 0.0), (W, H), (0.0, H), (CX, CY), (1234.5, 4321.0)])
def test_ray_flat_closed_form(u, v):
    R = A.R_NADIR @ A.rotvec_to_matrix(np.array([0.01, -0.02, 0.3]))
    T = np.array([3.0, -4.0, 300.0])
    d = G.pixel_ray(R, F, CX, CY, u, v)
    lam, st = G.ray_dsm(flat(20.0), T, d)
    assert st == 0
    assert abs(lam - (T[2] - 20.0) / -d[2]) < 1e-12 * lam


def test_ray_tilted_plane_closed_form():
    rng = np.random.default_rng(2)
    d_ = tilted()
    for _ in range(30):
        R = A.R_NADIR @ A.rotvec_to_matrix(rng.normal(0, 0.05, 3))
        T = np.array([rng.uniform(-50, 50), rng.uniform(-50, 50), 300.0])
        d = G.pixel_ray(R, F, CX, CY, rng.uniform(0, W), rng.uniform(0, H))
        lam, st = G.ray_dsm(d_, T, d)
        a, b, c = 0.125, -0.0625, 20.0
        ref = (a * T[0] + b * T[1] + c - T[2]) / (d[2] - a * d[0] - b * d[1])
        assert st == 0 and abs(lam - ref) < 1e-11 * ref


def test_ray_misses_when_not_descending():
    d = G.pixel_ray(np.eye(3), F, CX, CY, CX, CY)        # camera z axis = world up
    lam, st = G.ray_dsm(flat(), np.array([0.0, 0.0, 300.0]), d)
    assert st == G.MISS and math.isnan(lam)


def test_ray_hills_first_crossing_brute_force():
    g = hills()
    dsm = g["dsm"]
    rng = np.random.default_rng(3)
    for k in range(g["n_images"]):
        for u, v in [(0.0, 0.0), (W, H), (rng.uniform(0, W), rng.uniform(0, H))]:
            d = G.pixel_ray(g["R"][k], F, CX, CY, u, v)
            lam, st = G.ray_dsm(dsm, g["T"][k], d)
            assert st == 0
            X = g["T"][k] + lam * d
            assert abs(X[2] - G.dsm_height(dsm, X[0], X[1])) < 1e-9
            # brute force: no crossing before lam (steps of 1/100 cell of horizontal travel)
            step = 0.01 * dsm["cell"] / math.hypot(d[0], d[1])
            for t in np.arange(0.0, lam - 2 * step, step):
                P = g["T"][k] + t * d
                assert P[2] - G.dsm_height(dsm, P[0], P[1]) > 0.0


def test_footprint_nadir_flat_rectangle():
    R = A.R_NADIR
    T = np.array([10.0, 20.0, 320.0])
    fp, st = G.footprint(flat(20.0), R, T, F, CX, CY, W, H)
    assert st == 0
    s = 300.0 / F                      # metres per pixel at 300 m depth
    # camera x = world x, camera y = -world y (R_NADIR)
    ref = np.array([[10 - CX * s, 20 + CY * s, 20], [10 + CX * s, 20 + CY * s, 20], [10 + CX * s, 20 - CY * s, 20],
                    [10 - CX * s, 20 - CY * s, 20], [10, 20, 20]])
    assert np.abs(fp - ref).max() < 1e-9


def test_footprint_round_trip_through_generator_projection():
    g = hills()
    for k in range(g["n_images"]):
        fp, st = G.footprint(g["dsm"], g["R"][k], g["T"][k], F, CX, CY, W, H)
        assert st == 0
        uv, z = A.synth_project(g["R"][k][None], g["T"][k][None], fp, 0.0, 0.0)
        ref = np.array([[0, 0], [W, 0], [W, H], [0, H], [W / 2, H / 2]], float)
        assert np.abs(uv[:, 0, :] - ref).max() < 1e-6


def rect(x0, y0, x1, y1):
    return np.array([[x0, y0], [x1, y0], [x1, y1], [x0, y1]], float)


def test_overlap_closed_forms():
    assert G.overlap_area(rect(0, 0, 4, 3), rect(1, 1, 6, 2)) == pytest.approx(3.0, abs=1e-12)
    assert G.overlap_area(rect(0, 0, 4, 3), rect(5, 0, 6, 3)) == 0.0
    assert G.overlap_area(rect(0, 0, 10, 10), rect(2, 3, 4, 5)) == pytest.approx(4.0, abs=1e-12)
    assert G.overlap_area(rect(0, 0, 10, 10)[::-1], rect(2, 3, 4, 5)) == pytest.approx(4.0, abs=1e-12)
    s = 2.0
    sq = rect(-1, -1, 1, 1)
    c, sn = math.cos(math.pi / 4), math.sin(math.pi / 4)
    rot = sq @ np.array([[c, sn], [-sn, c]])
    assert G.overlap_area(sq, rot) == pytest.approx(2 * (math.sqrt(2) - 1) * s * s, rel=1e-12)


def test_overlap_dense_count_and_symmetry():
    rng = np.random.default_rng(4)
    g = hills()
    fps = [G.footprint(g["dsm"], g["R"][k], g["T"][k], F, CX, CY, W, H)[0] for k in range(g["n_images"])]
    for i, j in [(0, 1), (0, 2), (1, 7), (2, 9), (5, 6)]:
        a = G.overlap_area(fps[i][:4], fps[j][:4])
        assert a == pytest.approx(G.overlap_area(fps[j][:4], fps[i][:4]), rel=1e-12, abs=1e-9)
        # point-in-both count on a 1 m grid over the union's bounding box
        P = np.vstack([fps[i][:4, :2], fps[j][:4, :2]])
        xs = np.arange(P[:, 0].min(), P[:, 0].max(), 1.0) + 0.5
        ys = np.arange(P[:, 1].min(), P[:, 1].max(), 1.0) + 0.5
        X, Y = np.meshgrid(xs, ys)

        def inside(Q):
            Q = Q if G.polygon_area(Q) > 0 else Q[::-1]
            ok = np.ones_like(X, bool)
            for e in range(4):
                a_, b_ = Q[e], Q[(e + 1) % 4]
                ok &= (b_[0] - a_[0]) * (Y - a_[1]) - (b_[1] - a_[1]) * (X - a_[0]) >= 0
            return ok

        cnt = float((inside(fps[i][:4, :2]) & inside(fps[j][:4, :2])).sum())
        per = sum(np.hypot(*np.diff(np.vstack([q, q[:1]]), axis=0).T).sum() for q in (fps[i][:4, :2], fps[j][:4, :2]))
        assert abs(cnt - a) <= per + 1.0, (i, j, cnt, a)


def test_eq3_identity_and_translation():
    g = hills()
    uv0 = SG.patch_grid()[::37]
    R0, T0 = g["R"][0], g["T"][0]
    uv, lam, fl = G.transfer_eq3(g["dsm"], R0, T0, R0, T0, F, CX, CY, W, H, uv0)
    assert np.all(fl == 0) and np.abs(uv - uv0).max() < 1e-8
    # flat ground, same attitude, camera moved by t: shift = -(f / depth) R^T t (x, y of the camera frame)
    R = A.R_NADIR
    T0 = np.array([0.0, 0.0, 320.0])
    t = np.array([3.0, -7.5, 0.0])
    uv, lam, fl = G.transfer_eq3(flat(20.0), R, T0, R, T0 + t, F, CX, CY, W, H, uv0)
    shift = -(F / 300.0) * (R.T @ t)[:2]
    inner = fl == 0
    assert np.abs(uv[inner] - (uv0[inner] + shift)).max() < 1e-8


def test_eq3_matches_generator_projection_and_wraps():
    g = hills()
    uv0 = SG.patch_grid()
    R0, T0 = g["R"][0], g["T"][0]
    k = 3                                      # three base lengths along the strip: many patches leave
    uv, lam, fl = G.transfer_eq3(g["dsm"], R0, T0, g["R"][k], g["T"][k], F, CX, CY, W, H, uv0)
    assert np.all(fl != G.MISS)
    X = T0 + lam[:, None] * np.stack([G.pixel_ray(R0, F, CX, CY, u, v) for u, v in uv0])
    ref, _ = A.synth_project(g["R"][k][None], g["T"][k][None], X, 0.0, 0.0)
    ref = ref[:, 0, :]
    out = (ref[:, 0] < 0) | (ref[:, 0] >= W) | (ref[:, 1] < 0) | (ref[:, 1] >= H)
    assert out.any() and (~out).any()
    assert np.array_equal(fl == 2, out)
    assert np.abs(uv[~out] - ref[~out]).max() < 1e-6
    wrapped = np.stack([np.mod(ref[out, 0], W), np.mod(ref[out, 1], H)], 1)
    assert np.abs(uv[out] - wrapped).max() < 1e-6
