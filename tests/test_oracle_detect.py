"""Pins of the oracle's keypoint detector (FAST-9 score, suppression,
intensity-centroid orientation) against independent definitions and closed
forms: the segment test written out in numpy from a circle derived as the
lattice points at distance [2.5, 3.5), single-dot and constant images, linear
ramps with exactly known moments and angles, and quarter-turn invariance."""
import math

import numpy as np
import pytest

import oracle
from paper_1609_03986_amd import synth


def circle_offsets():
    pts = [(dx, dy) for dy in range(-3, 4) for dx in range(-3, 4)
           if 2.5 <= math.hypot(dx, dy) < 3.5]
    pts.sort(key=lambda p: math.atan2(p[1], p[0]))        # cyclic order
    assert len(pts) == 16
    return pts


def segment_test(img, x, y, t):
    """True iff 9 cyclically consecutive circle pixels are all > c + t or all < c - t."""
    c = int(img[y, x])
    ring = [int(img[y + dy, x + dx]) for dx, dy in circle_offsets()]
    for sign in (1, -1):
        ok = [sign * (v - c) > t for v in ring]
        for k in range(16):
            if all(ok[(k + j) % 16] for j in range(9)):
                return True
    return False


def test_score_is_the_largest_threshold_of_the_segment_test():
    g = np.random.default_rng(5)
    for trial in range(6):
        img = synth.smoothed_noise(g, 40, 40) if trial % 2 else g.integers(0, 256, (40, 40)).astype(np.uint8)
        for _ in range(60):
            x, y = (int(v) for v in g.integers(3, 37, 2))
            s = oracle.fast_score(img, x, y)
            for t in (0, 5, 20, 40, 80, s - 1, s, s + 1):
                if t < 0:
                    continue
                assert segment_test(img, x, y, t) == (s > t), (trial, x, y, t, s)


def test_single_dot_and_constant_image():
    img = np.full((64, 70), 30, np.uint8)
    kps, n = oracle.detect(img, 10)
    assert n == 0
    img[40, 33] = 230
    kps, n = oracle.detect(img, 10)
    assert n == 1 and kps[0, 0] == 33 and kps[0, 1] == 40 and kps[0, 3] == 1.0
    assert oracle.fast_score(img, 33, 40) == 200
    kps, n = oracle.detect(img, 200)            # score must exceed the threshold
    assert n == 0


def disc():
    r = oracle.ORIENT_RADIUS
    return [(dx, dy) for dy in range(-r, r + 1) for dx in range(-r, r + 1) if dx * dx + dy * dy <= r * r]


@pytest.mark.parametrize("ax,ay,bin_", [(1, 0, 0), (0, 1, 1024), (-1, 0, 2048), (0, -1, 3072),
                                        (1, 1, 512), (-1, 1, 1536)])
def test_orientation_of_ramps(ax, ay, bin_):
    h = w = 64
    yy, xx = np.mgrid[0:h, 0:w]
    img = (128 + 2 * ax * (xx - 32) + 2 * ay * (yy - 32)).astype(np.uint8)
    b, m10, m01 = oracle.orientation_bin(img, 32, 32)
    d = disc()
    want10 = sum(dx * int(img[32 + dy, 32 + dx]) for dx, dy in d)
    want01 = sum(dy * int(img[32 + dy, 32 + dx]) for dx, dy in d)
    assert (m10, m01) == (want10, want01)
    assert m10 == 2 * ax * sum(dx * dx for dx, dy in d) and m01 == 2 * ay * sum(dy * dy for dx, dy in d)
    assert b == bin_


def test_orientation_matches_textbook_angle():
    g = np.random.default_rng(9)
    img = synth.smoothed_noise(g, 80, 80)
    for _ in range(50):
        x, y = (int(v) for v in g.integers(16, 64, 2))
        b, m10, m01 = oracle.orientation_bin(img, x, y)
        ang = math.degrees(math.atan2(m01, m10)) % 360.0
        assert abs(((b * 360.0 / 4096.0 - ang) + 180.0) % 360.0 - 180.0) <= 360.0 / 4096.0 / 2 + 1e-9


def test_quarter_turn_invariance():
    g = np.random.default_rng(17)
    n = 160
    img = synth.smoothed_noise(g, n, n)
    kps, cnt = oracle.detect(img, 20)
    assert cnt > 200
    rot = np.ascontiguousarray(np.rot90(img))             # rot[i][j] = img[j][n - 1 - i]
    kr, cr = oracle.detect(rot, 20)
    assert cr == cnt
    bins = np.rint(kps[:, 2] * 4096.0 / 360.0).astype(int)
    mapped = {(int(y), n - 1 - int(x), int((b - 1024) % 4096)) for (x, y, _, _), b in zip(kps, bins)}
    got = {(int(x), int(y), int(np.rint(a * 4096.0 / 360.0)) % 4096) for x, y, a, _ in kr}
    assert got == mapped


def test_raster_order_and_truncation():
    g = np.random.default_rng(21)
    img = synth.smoothed_noise(g, 120, 200)
    kps, n = oracle.detect(img, 15)
    assert n > 100
    order = kps[:, 1] * 10000 + kps[:, 0]
    assert np.all(np.diff(order) > 0)
    k5, n5 = oracle.detect(img, 15, max_kps=5)
    assert n5 == n and np.array_equal(k5, kps[:5])


def test_orientation_bin_does_not_depend_on_last_bits_of_atan2():
    """The moments are integers of magnitude at most M, so their angle keeps a
    distance from every bin boundary (2k + 1) pi / 4096 that is far above the
    error of a double atan2 and product: any atan2 accurate to a few ulp gives
    the same bin.  The closest approach is found from the continued fraction of
    tan of each boundary in the first octant (the boundaries are symmetric
    under reflection in the axes and the diagonal), whose convergents and
    largest admissible semiconvergents are the best approximations p / q with
    q <= M."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 60
    r = oracle.ORIENT_RADIUS
    M = 255 * sum(abs(dx) for dy in range(-r, r + 1) for dx in range(-r, r + 1)
                  if dx * dx + dy * dy <= r * r)
    C = mpmath.mpf(4096) / (2 * mpmath.pi)
    worst = mpmath.mpf(1)
    for k in range(512):                          # boundaries in (0, pi / 4)
        t = mpmath.tan((2 * k + 1) * mpmath.pi / 4096)
        cands = []
        p0, q0, p1, q1 = 0, 1, 1, 0               # convergents p_{n-1}/q_{n-1}, p_n/q_n
        x = t
        while True:
            a = int(mpmath.floor(x))
            p2, q2 = a * p1 + p0, a * q1 + q0
            if q2 > M:
                j = (M - q0) // q1                # largest semiconvergent within M
                if j >= 1:
                    cands.append((j * p1 + p0, j * q1 + q0))
                break
            cands.append((p2, q2))
            p0, q0, p1, q1 = p1, q1, p2, q2
            frac = x - a
            if frac == 0:
                break
            x = 1 / frac
        for p, q in cands:
            if q == 0:
                continue
            d = abs(mpmath.atan(mpmath.mpf(p) / q) * C - (k + mpmath.mpf(1) / 2))
            worst = min(worst, d)
    # Error of the computed rint argument for |atan2| <= pi: atan2 within 4
    # ulp (of pi: 2^-51 each), the double constant 4096 / 2 pi and the product
    # each rounded (relative 2^-53 of at most 2048).
    err = 4 * 2.0 ** -51 * float(C) + 2 * 2048 * 2.0 ** -53
    assert M < 1 << 21
    assert worst > 2 * err, (float(worst), err)


# --- Suppression and border (the rule of the detector, as the library fixes it:
# keep a corner whose score is strictly above every corner among its 8
# neighbours, and test only pixels at least 16 from every edge). ---

def numpy_scores(img):
    """FAST-9 score of every pixel whose circle fits, from the lattice circle:
    per pixel, the largest over the 16 arcs of 9 and both polarities of the
    smallest difference on the arc.  Pixels whose circle leaves the image get
    -256 (never a corner)."""
    h, w = img.shape
    a = img.astype(np.int32)
    ring = np.stack([np.roll(np.roll(a, -dy, 0), -dx, 1) for dx, dy in circle_offsets()])
    best = np.full((h, w), -256, np.int32)
    for sign in (1, -1):
        d = sign * (ring - a[None])
        for k in range(16):
            arc = d[[(k + j) % 16 for j in range(9)]].min(axis=0)
            best = np.maximum(best, arc)
    best[:3, :] = best[-3:, :] = -256
    best[:, :3] = best[:, -3:] = -256
    return best


def numpy_detect_positions(img, t, border=16):
    """Raster-ordered (x, y) of the corners that survive strict 8-neighbour
    suppression, brute force."""
    h, w = img.shape
    s = numpy_scores(img)
    S = np.zeros((h, w), np.int64)
    inside = np.zeros((h, w), bool)
    inside[border:h - border, border:w - border] = True
    S[inside & (s > t)] = s[inside & (s > t)]
    out = []
    for y in range(h):
        for x in range(w):
            if S[y, x] <= 0:
                continue
            nb = [S[y + dy, x + dx] for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                  if (dx or dy) and 0 <= y + dy < h and 0 <= x + dx < w]
            if all(S[y, x] > v for v in nb):
                out.append((x, y))
    return out


def positions(kps):
    return [(int(x), int(y)) for x, y, _, _ in kps]


@pytest.mark.parametrize("shape,t,seed", [((48, 60), 10, 1), ((64, 70), 20, 2), ((33, 33), 5, 3),
                                          ((40, 90), 15, 4), ((70, 41), 0, 5)])
def test_detect_equals_brute_force_suppression(shape, t, seed):
    g = np.random.default_rng(seed)
    img = g.integers(0, 256, shape).astype(np.uint8) if seed % 2 else synth.smoothed_noise(g, *shape)
    kps, n = oracle.detect(img, t)
    want = numpy_detect_positions(img, t)
    assert n == len(want) and positions(kps) == want


def dots(shape, pts, background=30):
    img = np.full(shape, background, np.uint8)
    for x, y, v in pts:
        img[y, x] = v
    return img


def test_equal_adjacent_corners_suppress_each_other():
    # Two bright dots side by side: each has score 200, and neither lies on
    # the other's circle, so the plateau keeps neither.
    img = dots((64, 70), [(33, 40, 230), (34, 40, 230)])
    assert oracle.fast_score(img, 33, 40) == 200 and oracle.fast_score(img, 34, 40) == 200
    assert oracle.detect(img, 10)[1] == 0
    # The same vertically.
    assert oracle.detect(dots((64, 70), [(33, 40, 230), (33, 41, 230)]), 10)[1] == 0


def test_corner_beside_a_stronger_one_is_dropped():
    img = dots((64, 70), [(33, 40, 230), (34, 40, 200)])     # scores 200 and 170
    kps, n = oracle.detect(img, 10)
    assert n == 1 and positions(kps) == [(33, 40)]
    img = dots((64, 70), [(33, 40, 180), (33, 41, 230)])
    kps, n = oracle.detect(img, 10)
    assert n == 1 and positions(kps) == [(33, 41)]


@pytest.mark.parametrize("d", [(1, 1), (-1, 1), (1, -1), (-1, -1)])
def test_diagonal_neighbours_take_part_in_suppression(d):
    # A 4-neighbourhood would keep both dots.
    x, y = 33, 40
    img = dots((64, 70), [(x, y, 230), (x + d[0], y + d[1], 200)])
    kps, n = oracle.detect(img, 10)
    assert n == 1 and positions(kps) == [(x, y)]
    img = dots((64, 70), [(x, y, 230), (x + d[0], y + d[1], 230)])
    assert oracle.detect(img, 10)[1] == 0


def test_two_pixels_apart_both_survive():
    img = dots((64, 70), [(33, 40, 230), (35, 40, 200)])
    kps, n = oracle.detect(img, 10)
    assert n == 2 and positions(kps) == [(33, 40), (35, 40)]


@pytest.mark.parametrize("h,w", [(64, 70), (50, 41)])
def test_border_of_sixteen_pixels(h, w):
    # A dot is kept iff it is at least 16 pixels from every edge: columns
    # 16 .. w - 17 and rows 16 .. h - 17.
    cases = [((16, 24), True), ((15, 24), False), ((w - 17, 24), True), ((w - 16, 24), False),
             ((20, 16), True), ((20, 15), False), ((20, h - 17), True), ((20, h - 16), False)]
    for (x, y), kept in cases:
        kps, n = oracle.detect(dots((h, w), [(x, y, 230)]), 10)
        assert n == (1 if kept else 0), (x, y)
        if kept:
            assert positions(kps) == [(x, y)]


def test_smallest_images():
    # 33 x 33 has exactly one pixel 16 from every edge; 32 x 32 has none.
    kps, n = oracle.detect(dots((33, 33), [(16, 16, 230)]), 10)
    assert n == 1 and positions(kps) == [(16, 16)]
    assert oracle.detect(dots((32, 32), [(16, 16, 230)]), 10)[1] == 0
    assert oracle.detect(dots((32, 32), [(15, 15, 230)]), 10)[1] == 0
    for h, w in [(33, 32), (32, 33), (1, 1), (16, 200)]:
        assert oracle.detect(np.full((h, w), 77, np.uint8), 0)[1] == 0
