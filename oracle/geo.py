"""FP64 CPU oracle of the image footprints, their overlaps and the GNSS/IMU
patch transfer (Sec. 3.1, Eq. 3) (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  Plain numpy and Python loops, written from the paper and
the readings below; it shares nothing with the HIP library.

Readings (the paper names the operations, not their numerics):
* DSM: heights on raster nodes (x0 + i cell, y0 + j cell); between nodes the
  surface is the bilinear interpolation of the four surrounding nodes;
  outside the raster the position is clamped to it.
* Pixel ray (Eq. 3): X(lam) = T + lam R K^-1 (u, v, 1)^T, so lam is the depth
  along the camera axis, as Eq. 3's nominal depth.
* Ray / DSM intersection: the first lam > 0 where the ray's height meets the
  surface, g(lam) = z(lam) - H(x(lam), y(lam)) = 0.  The ray is sampled from
  where it passes the raster's highest node to where it passes the lowest,
  in n equal steps, n = ceil(horizontal travel / half a cell), at least 1
  and at most 65536;
  the first sample with g <= 0 and the one before it bracket the root,
  which up to 64 halvings then narrow (the root is the bracket's final
  upper end).  A ray that does not descend misses.
* Footprint (Sec. 3.1): the ground points of the four image corners
  (0, 0), (W, 0), (W, H), (0, H) and of the image centre (W/2, H/2).
* Overlap of two footprints: the area of the intersection of their corner
  quadrilaterals in the horizontal plane (both convex).
* Eq. 3 with an a-priori elevation model: lam of the patch centre's ray in
  image 0 is its DSM intersection; the ground point is projected into image
  k with K and (R_k, T_k) (a ground point not in front of camera k counts
  as a miss).  A patch whose centre leaves the image
  [0, W) x [0, H) re-enters at the opposite edge (Sec. 3.1): the coordinate
  is wrapped modulo the image size, and the patch is flagged.
"""
from __future__ import annotations

import math

import numpy as np

MISS = 1        # ray does not meet the DSM (it does not descend, or passes below nothing)


def dsm_height(dsm: dict, x: float, y: float) -> float:
    """Bilinear height of the raster at (x, y), position clamped to the raster."""
    nx, ny, cell = dsm["nx"], dsm["ny"], dsm["cell"]
    h = dsm["h"]
    gx = min(max((x - dsm["x0"]) / cell, 0.0), nx - 1.0)
    gy = min(max((y - dsm["y0"]) / cell, 0.0), ny - 1.0)
    i = min(int(math.floor(gx)), nx - 2)
    j = min(int(math.floor(gy)), ny - 2)
    fx, fy = gx - i, gy - j
    h00, h10 = float(h[j, i]), float(h[j, i + 1])
    h01, h11 = float(h[j + 1, i]), float(h[j + 1, i + 1])
    return (1 - fx) * (1 - fy) * h00 + fx * (1 - fy) * h10 + (1 - fx) * fy * h01 + fx * fy * h11


def pixel_ray(R, f, cx, cy, u, v) -> np.ndarray:
    """World direction R K^-1 (u, v, 1): lam along it is the camera-frame depth."""
    return np.asarray(R, np.float64) @ np.array([(u - cx) / f, (v - cy) / f, 1.0])


def ray_dsm(dsm: dict, T, d):
    """(lam, status) of the first intersection of T + lam d with the DSM."""
    T = np.asarray(T, np.float64)
    d = np.asarray(d, np.float64)
    if not d[2] < 0.0:
        return math.nan, MISS
    hmin, hmax = float(np.min(dsm["h"])), float(np.max(dsm["h"]))
    lam_a = max(0.0, (T[2] - hmax) / -d[2])
    lam_b = (T[2] - hmin) / -d[2]
    if not lam_b > 0.0:
        return math.nan, MISS

    def g(lam):
        return T[2] + lam * d[2] - dsm_height(dsm, T[0] + lam * d[0], T[1] + lam * d[1])

    if g(lam_a) <= 0.0:
        return lam_a, 0
    dxy = math.hypot(d[0], d[1])
    n = 1 if dxy == 0.0 else min(65536, max(1, int(math.ceil((lam_b - lam_a) * dxy / (0.5 * dsm["cell"])))))
    lo = lam_a
    hi = lam_b
    for i in range(1, n + 1):
        lam = lam_b if i == n else lam_a + (lam_b - lam_a) * i / n
        if g(lam) <= 0.0:
            hi = lam
            break
        lo = lam
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if g(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return hi, 0


def footprint(dsm: dict, R, T, f, cx, cy, width, height):
    """Ground points [5][3] of the corners (0,0), (W,0), (W,H), (0,H) and the
    centre (W/2, H/2), and a status (MISS if any ray misses)."""
    out = np.full((5, 3), np.nan)
    status = 0
    for c, (u, v) in enumerate([(0.0, 0.0), (width, 0.0), (width, height), (0.0, height),
                                (0.5 * width, 0.5 * height)]):
        d = pixel_ray(R, f, cx, cy, u, v)
        lam, st = ray_dsm(dsm, T, d)
        if st:
            status = MISS
            continue
        out[c] = np.asarray(T, np.float64) + lam * d
    return out, status


def polygon_area(P) -> float:
    """Signed (counter-clockwise positive) area by the shoelace formula."""
    P = np.asarray(P, np.float64)
    x, y = P[:, 0], P[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def _is_convex_ccw(P) -> bool:
    n = len(P)
    for i in range(n):
        a, b, c = P[i], P[(i + 1) % n], P[(i + 2) % n]
        if (b[0] - a[0]) * (c[1] - b[1]) - (b[1] - a[1]) * (c[0] - b[0]) < 0.0:
            return False
    return True


def clip_convex(subject, clip):
    """Sutherland-Hodgman: the part of polygon `subject` inside the convex,
    counter-clockwise polygon `clip`."""
    out = [np.asarray(p, np.float64) for p in subject]
    m = len(clip)
    for e in range(m):
        a, b = np.asarray(clip[e], np.float64), np.asarray(clip[(e + 1) % m], np.float64)
        side = lambda p: (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])
        inp, out = out, []
        if not inp:
            break
        for i in range(len(inp)):
            p, q = inp[i], inp[(i + 1) % len(inp)]
            sp, sq = side(p), side(q)
            if sp >= 0.0:
                out.append(p)
            if (sp >= 0.0) != (sq >= 0.0):
                out.append(p + (q - p) * (sp / (sp - sq)))
    return out


def overlap_area(A, B) -> float:
    """Area of the intersection of two convex quadrilaterals (x, y)."""
    A = np.asarray(A, np.float64)[:, :2]
    B = np.asarray(B, np.float64)[:, :2]
    if polygon_area(A) < 0:
        A = A[::-1]
    if polygon_area(B) < 0:
        B = B[::-1]
    if not (_is_convex_ccw(A) and _is_convex_ccw(B)):
        raise ValueError("footprint quadrilateral is not convex")
    P = clip_convex(A, B)
    return abs(polygon_area(np.array(P))) if len(P) >= 3 else 0.0


def overlaps(fp) -> np.ndarray:
    """Packed upper triangle (i < j, row-major) of the pairwise overlap areas
    of footprints fp [n][5][3] (corners 0..3)."""
    n = len(fp)
    out = []
    for i in range(n):
        for j in range(i + 1, n):
            out.append(overlap_area(fp[i][:4], fp[j][:4]))
    return np.array(out)


def transfer_eq3(dsm: dict, R0, T0, Rk, Tk, f, cx, cy, width, height, uv0):
    """Eq. (3) for each patch centre uv0 [n][2] of image 0 into image k.
    Returns (uv [n][2] after re-initialisation, lam [n], flags [n]): flag 1 =
    the ray missed the DSM (uv NaN), 2 = re-initialised at the opposite edge."""
    n = len(uv0)
    uv = np.full((n, 2), np.nan)
    lam_out = np.full(n, np.nan)
    flags = np.zeros(n, np.int32)
    Rk = np.asarray(Rk, np.float64)
    for p in range(n):
        u0, v0 = uv0[p]
        d = pixel_ray(R0, f, cx, cy, u0, v0)
        lam, st = ray_dsm(dsm, T0, d)
        if st:
            flags[p] = MISS
            continue
        X = np.asarray(T0, np.float64) + lam * d
        xc = Rk.T @ (X - np.asarray(Tk, np.float64))
        if not xc[2] > 0.0:
            flags[p] = MISS
            continue
        u = f * xc[0] / xc[2] + cx
        v = f * xc[1] / xc[2] + cy
        if not (0.0 <= u < width and 0.0 <= v < height):
            u -= width * math.floor(u / width)
            v -= height * math.floor(v / height)
            flags[p] = 2
        uv[p] = (u, v)
        lam_out[p] = lam
    return uv, lam_out, flags


def _quad_ok(q) -> bool:
    q = np.asarray(q, np.float64)[:4, :2]
    if not np.all(np.isfinite(q)):
        return False
    if polygon_area(q) < 0:
        q = q[::-1]
    return _is_convex_ccw(q)


def cluster_membership(fp, strip, max_back=7, free_back=3, max_cams=20, min_cams=8, min_overlap=0.05):
    """The images of the cluster each image triggers (Sec. 3.1: overlapping
    images, within and across strips, are found by comparing footprints;
    Sec. 3.2: the cluster of the current image and its overlapping images,
    the part already adjusted held fixed).  fp [n][5][3] footprints in
    flight order, strip [n] the strip of each image.

    Two images overlap when both footprints exist (finite, convex corner
    quadrilaterals and a finite centre point) and the area of their intersection is at least
    min_overlap times the smaller of the two footprint areas.  The cluster
    of image i: i; then its in-strip predecessors i-1, i-2, ... (at most
    max_back, same strip, each overlapping the image after it); then the
    earlier images of other strips that overlap image i, nearest first by
    the horizontal distance of the footprint centres (ties: lower index);
    the list cut at max_cams.  Fewer than min_cams images: no cluster.
    Fixed: the earlier images of other strips and the in-strip predecessors
    more than free_back steps back; free: i and the rest.

    Returns, per image, None or (members ascending, fixed flags aligned)."""
    n = len(fp)
    strip = np.asarray(strip)
    ok = [_quad_ok(fp[k]) and bool(np.all(np.isfinite(np.asarray(fp[k], np.float64)[4, :2]))) for k in range(n)]
    area = [abs(polygon_area(np.asarray(fp[k], np.float64)[:4, :2])) if ok[k] else 0.0 for k in range(n)]

    def overlapping(a, b):
        if not (ok[a] and ok[b]):
            return False
        return overlap_area(fp[a][:4], fp[b][:4]) >= min_overlap * min(area[a], area[b])

    out = []
    for i in range(n):
        own = []
        j = i - 1
        while j >= 0 and len(own) < max_back and strip[j] == strip[i] and overlapping(j, j + 1):
            own.append(j)
            j -= 1
        cand = []
        for j in range(i):
            if strip[j] != strip[i] and overlapping(i, j):
                dx = fp[j][4][0] - fp[i][4][0]
                dy = fp[j][4][1] - fp[i][4][1]
                cand.append((dx * dx + dy * dy, j))
        cand.sort()
        cams = ([i] + own + [j for _, j in cand])[:max_cams]
        if len(cams) < min_cams:
            out.append(None)
            continue
        cams = sorted(cams)
        fixed = [0 if (k == i or (strip[k] == strip[i] and i - k <= free_back)) else 1 for k in cams]
        out.append((np.array(cams, np.int32), np.array(fixed, np.uint8)))
    return out
