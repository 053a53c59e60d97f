"""Pins of the oracle's cluster membership (oracle/geo.py
cluster_membership): the rule that turns footprints into the images of the
cluster each new image triggers (Sec. 3.1: overlapping images within and
across strips are found by comparing footprints; Sec. 3.2: the cluster of
the current image and its overlapping images, the part adjusted before held
fixed).

Footprints here are axis-aligned rectangles laid out by hand, so every
overlap area and every distance is a closed form, and the expected clusters
are written out from the rule's statement."""
import numpy as np
import pytest

from oracle import geo as OG


def rect(cx, cy, w, h):
    """Footprint [5][3]: corners (counter-clockwise) and centre of a w x h rectangle."""
    return np.array([[cx - w / 2, cy - h / 2, 0.0], [cx + w / 2, cy - h / 2, 0.0], [cx + w / 2, cy + h / 2, 0.0],
                     [cx - w / 2, cy + h / 2, 0.0], [cx, cy, 0.0]])


def strip_flight(n_strips, per, base, spacing, w=100.0, h=80.0):
    """Boustrophedon flight of rectangles: strip s at x = s spacing, images
    base apart along y (flown back on odd strips); flight order."""
    fp, strip = [], []
    for s in range(n_strips):
        for i in range(per):
            y = i * base if s % 2 == 0 else (per - 1 - i) * base
            fp.append(rect(s * spacing, y, w, h))
            strip.append(s)
    return np.array(fp), np.array(strip, np.int32)


def test_single_strip_sliding_window():
    """One strip, images 16 m apart with 80 m footprints: consecutive images
    overlap by 64/80, so the in-strip chain runs back max_back images; the
    cluster of image i is i and min(i, max_back) predecessors."""
    fp, strip = strip_flight(1, 12, 16.0, 0.0)
    out = OG.cluster_membership(fp, strip, max_back=7, free_back=3, max_cams=20, min_cams=5, min_overlap=0.05)
    for i, m in enumerate(out):
        if i < 4:
            assert m is None                      # fewer than 5 images
            continue
        cams, fixed = m
        lo = max(0, i - 7)
        assert cams.tolist() == list(range(lo, i + 1))
        assert fixed.tolist() == [1 if i - k > 3 else 0 for k in range(lo, i + 1)]


def test_chain_breaks_where_consecutive_images_do_not_overlap():
    """Images 16 m apart, then a 200 m jump after image 5: the chain of
    image 8 stops at image 6 (6 does not overlap 5)."""
    fp, strip = strip_flight(1, 10, 16.0, 0.0)
    fp[6:, :, 1] += 200.0
    out = OG.cluster_membership(fp, strip, max_back=7, free_back=3, max_cams=20, min_cams=1, min_overlap=0.05)
    assert out[8][0].tolist() == [6, 7, 8]
    assert out[5][0].tolist() == [0, 1, 2, 3, 4, 5]


def test_threshold_on_the_smaller_footprint():
    """Image 1 overlaps image 0 by 4 m x 80 m = 320 m^2 = 4 % of the 8000 m^2
    footprint: not overlapping at min_overlap 0.05, overlapping at 0.03."""
    fp = np.array([rect(0, 0, 100, 80), rect(96, 0, 100, 80)])
    strip = np.array([0, 1], np.int32)
    a = OG.cluster_membership(fp, strip, min_cams=1, min_overlap=0.05)
    b = OG.cluster_membership(fp, strip, min_cams=1, min_overlap=0.03)
    assert a[1][0].tolist() == [1] and b[1][0].tolist() == [0, 1]
    assert b[1][1].tolist() == [1, 0]             # the other strip's image is fixed


def test_cross_strip_nearest_first_with_cap():
    """Two strips 60 m apart (40 % side overlap of the 100 m width), images
    16 m apart; image 12 (second strip, flown back, at y = 3*16 = 48 m) sees
    the first strip's images whose rectangles overlap it, taken nearest
    first by centre distance sqrt(60^2 + dy^2): dy = 0 (image 3), then
    16 m (2 and 4, tie broken by index: 2 first), then 32 m (1, 5)...  With
    max_cams 6 and one in-strip predecessor allowed (image 11) the cluster
    is 12, 11, then 3, 2, 4, 1."""
    fp, strip = strip_flight(2, 8, 16.0, 60.0)
    out = OG.cluster_membership(fp, strip, max_back=1, free_back=3, max_cams=6, min_cams=1, min_overlap=0.05)
    cams, fixed = out[12]
    assert cams.tolist() == [1, 2, 3, 4, 11, 12]
    assert fixed.tolist() == [1, 1, 1, 1, 0, 0]
    # uncapped: every first-strip image within 80 m along y (overlap > 0) and above 5 %: dy < 80 (1 - 0.05 / 0.4)
    full = OG.cluster_membership(fp, strip, max_back=7, free_back=3, max_cams=64, min_cams=1, min_overlap=0.05)
    own = [11, 10, 9, 8]                           # images 8..11 precede 12 in its strip
    dy = np.abs(np.arange(8) * 16.0 - 48.0)
    ov = 40.0 * np.clip(80.0 - dy, 0.0, None)
    cross = [j for j in range(8) if ov[j] >= 0.05 * 8000.0]
    assert full[12][0].tolist() == sorted(own + cross + [12])


def test_missing_footprint_neither_joins_nor_triggers_across():
    fp, strip = strip_flight(2, 4, 16.0, 60.0)
    fp[1, 0] = np.nan                              # a corner ray of image 1 missed the DSM
    out = OG.cluster_membership(fp, strip, max_back=7, free_back=3, max_cams=20, min_cams=1, min_overlap=0.05)
    assert 1 not in out[6][0].tolist()             # not a cross-strip member
    assert out[2][0].tolist() == [2]               # the chain of image 2 stops at image 1
    assert out[1][0].tolist() == [1]               # it triggers a cluster of itself alone
