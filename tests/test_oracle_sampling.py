"""Pins for the oracle's window resampling (rule R) and rotation table.

The paper (Sec. 3.2, "Memory optimization") resamples the rotated window of an
oriented keypoint into an upright square but does not state the sampling; the
oracle fixes rule R.  These tests pin it to things other than itself: numpy
crops and edge padding, the textbook rotation matrix, closed forms for quarter
turns and integer scales, and the values of cos/sin.
"""
import numpy as np
import pytest

import oracle

W = oracle.WINDOW


def coord_images(h=256, w=256):
    """Two images whose pixel values are their own x and y coordinates."""
    yy, xx = np.mgrid[0:h, 0:w]
    return (xx & 255).astype(np.uint8), (yy & 255).astype(np.uint8)


def test_rotation_table_fixed_points():
    c, s = oracle.rotation_table()
    assert (c[0], s[0]) == (16384, 0)
    assert (c[512], s[512]) == (11585, 11585)          # 16384 / sqrt(2) = 11585.24
    assert (c[1024], s[1024]) == (0, 16384)
    assert (c[2048], s[2048]) == (-16384, 0)
    assert (c[3072], s[3072]) == (0, -16384)


def test_rotation_table_matches_cos_sin_and_quarter_turn_symmetry():
    c, s = oracle.rotation_table()
    a = np.arange(4096)
    th = 2 * np.pi * a / 4096
    assert np.max(np.abs(c - 16384 * np.cos(th))) <= 0.5 + 1e-9
    assert np.max(np.abs(s - 16384 * np.sin(th))) <= 0.5 + 1e-9
    # Quarter turn (C, S) -> (-S, C) holds exactly for every bin.
    assert np.array_equal(np.roll(c, -1024), -s)
    assert np.array_equal(np.roll(s, -1024), c)
    # Reflection about 45 degrees inside the first quadrant.
    assert np.array_equal(c[1:1024][::-1], s[1:1024])


def test_rotation_table_entries_are_far_from_rounding_ties():
    # Every rounded value of the first octant sits well away from a .5 tie,
    # so any correct double evaluation of cos/sin gives the same table.
    a = np.arange(513)
    for v in (16384 * np.cos(2 * np.pi * a / 4096), 16384 * np.sin(2 * np.pi * a / 4096)):
        frac = np.abs(v - np.floor(v) - 0.5)
        assert frac.min() > 1e-6


def test_upright_unit_scale_is_a_plain_crop():
    g = np.random.default_rng(5)
    img = g.integers(0, 256, size=(120, 160), dtype=np.uint8)
    for x, y in [(80.0, 60.0), (80.49, 60.2), (79.5, 59.5), (30.0, 30.0)]:
        cx, cy = int(np.floor(x + 0.5)), int(np.floor(y + 0.5))
        tile, f = oracle.sample_window(img, x, y, 0.0, 1.0)
        assert f == 0
        assert np.array_equal(tile, img[cy - 24:cy + 24, cx - 24:cx + 24])


def test_centre_rounding_is_half_up_in_double():
    ix, iy = coord_images()
    # 0.5 - 2^-25 is a float32 whose float32 sum with 0.5 rounds to 1.0, but
    # floor(x + 0.5) evaluated in double is 0.
    x = float(np.float32(0.5) - np.float32(2.0 ** -25))
    assert np.float32(x) == x
    for xv, want in [(x, 0), (100.5, 101), (99.5, 100), (100.49999, 100), (-0.5, 0),
                     (-0.51, -1), (-1.5, -1)]:
        assert float(np.float32(xv)) == xv or xv in (100.49999, -0.51)
        tile, f = oracle.sample_window(ix, xv, 128.0)
        assert f == 0
        # column 26 of the upright unit-scale tile samples x = cx + 2 exactly.
        assert int(tile[24, 26]) == want + 2, xv


def test_quarter_turns_closed_form():
    ix, iy = coord_images()
    cx, cy = 128, 100
    i, j = np.mgrid[0:W, 0:W]
    u, v = j - 24, i - 24
    cases = {
        90.0: (-v, u),      # R(90) (u, v) = (-v, u)
        180.0: (-u, -v),
        270.0: (v, -u),
        -90.0: (v, -u),
        450.0: (-v, u),
    }
    for ang, (ox, oy) in cases.items():
        tx, _ = oracle.sample_window(ix, cx, cy, ang, 1.0)
        ty, _ = oracle.sample_window(iy, cx, cy, ang, 1.0)
        assert np.array_equal(tx.astype(int), cx + ox), ang
        assert np.array_equal(ty.astype(int), cy + oy), ang


def test_integer_scale_upright_closed_form():
    ix, iy = coord_images()
    i, j = np.mgrid[0:W, 0:W]
    for sc in (2.0, 0.5, 1.25):
        tx, _ = oracle.sample_window(ix, 128, 128, 0.0, sc)
        ty, _ = oracle.sample_window(iy, 128, 128, 0.0, sc)
        # sc * u is an exact multiple of 1/4; half away from zero on ties.
        want_x = 128 + np.sign(sc * (j - 24)) * np.floor(np.abs(sc * (j - 24)) + 0.5)
        want_y = 128 + np.sign(sc * (i - 24)) * np.floor(np.abs(sc * (i - 24)) + 0.5)
        assert np.array_equal(tx.astype(int), want_x.astype(int)), sc
        assert np.array_equal(ty.astype(int), want_y.astype(int)), sc


@pytest.mark.parametrize("seed", range(6))
def test_matches_textbook_rotation_away_from_ties(seed):
    """Offsets equal round(s R(theta) (u, v)) with libm cos/sin, except where the
    exact value is within the Q14 table's own error of a rounding tie."""
    g = np.random.default_rng(100 + seed)
    ix, iy = coord_images()
    i, j = np.mgrid[0:W, 0:W]
    u, v = j - 24.0, i - 24.0
    for _ in range(20):
        b = int(g.integers(0, 4096))
        ang = b * 45.0 / 512.0                     # exactly bin b
        sc = float(g.choice([0.6, 1.0, 1.2, 1.44, 1.728, 2.0736]))
        th = 2 * np.pi * b / 4096
        sq = np.rint(sc * 256) / 256
        fx = sq * (np.cos(th) * u - np.sin(th) * v)
        fy = sq * (np.sin(th) * u + np.cos(th) * v)
        tx, f1 = oracle.sample_window(ix, 128, 128, np.float32(ang), sc)
        ty, f2 = oracle.sample_window(iy, 128, 128, np.float32(ang), sc)
        assert f1 == 0 and f2 == 0
        ox, oy = tx.astype(int) - 128, ty.astype(int) - 128
        rx = np.sign(fx) * np.floor(np.abs(fx) + 0.5)
        ry = np.sign(fy) * np.floor(np.abs(fy) + 0.5)
        # Q14 table error is <= 0.5/16384 per unit; margin covers |u|,|v| <= 24 at scale <= 2.1.
        safe_x = np.abs(np.abs(fx) - np.floor(np.abs(fx)) - 0.5) > 5e-3
        safe_y = np.abs(np.abs(fy) - np.floor(np.abs(fy)) - 0.5) > 5e-3
        assert np.array_equal(ox[safe_x], rx[safe_x]), (b, sc)
        assert np.array_equal(oy[safe_y], ry[safe_y]), (b, sc)
        assert safe_x.mean() > 0.9 and safe_y.mean() > 0.9


def test_border_clamp_is_edge_replication():
    g = np.random.default_rng(9)
    img = g.integers(0, 256, size=(60, 70), dtype=np.uint8)
    padded = np.pad(img, 64, mode="edge")
    for x, y in [(0, 0), (69, 59), (3, 50), (-10, -20), (100, 5)]:
        tile, f = oracle.sample_window(img, x, y, 0.0, 1.0)
        assert f == 0
        cx, cy = x + 64, y + 64
        assert np.array_equal(tile, padded[cy - 24:cy + 24, cx - 24:cx + 24]), (x, y)


def test_bin_exact_angles_map_to_their_bins():
    ix, iy = coord_images()
    c, s = oracle.rotation_table()
    for b in [0, 1, 2, 511, 512, 513, 1023, 1024, 2047, 3000, 4095]:
        tx, _ = oracle.sample_window(ix, 128, 128, b * 45.0 / 512.0, 1.0)
        # window pixel (i=24, j=47): u = 23, v = 0 -> ox = round(23 C / 16384)
        cb = int(c[b])
        want = 128 + int(np.sign(cb) * np.floor(abs(23 * cb) / 16384 + 0.5))
        assert int(tx[24, 47]) == want, b


def test_out_of_domain_keypoints_are_flagged():
    img = np.zeros((64, 64), np.uint8)
    bad = [(np.nan, 1, 0, 1), (1, np.inf, 0, 1), (1, 1, np.nan, 1), (1, 1, 0, np.nan),
           (1, 1, 1.5e6, 1), (1, 1, 0, 0.0), (1, 1, 0, 1.0 / 1024), (1, 1, 0, 5.0),
           (1, 1, 0, -1.0), (3e7, 1, 0, 1)]
    for kp in bad:
        _, f = oracle.sample_window(img, *kp)
        assert f == oracle.FLAG_BAD_KEYPOINT, kp
    good = [(1, 1, 0, 1.0 / 256), (1, 1, 0, 4.0), (1, 1, -1e6, 1), (-1e5, 2e5, 10, 1)]
    for kp in good:
        _, f = oracle.sample_window(img, *kp)
        assert f == 0, kp
