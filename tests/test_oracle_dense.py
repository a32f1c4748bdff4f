"""Pins of the oracle's dense CLATCH and windowed dense matching (Sec. 6):
dense descriptors are extraction at every pixel (upright, scale 1), which
equals a numpy box-filter formulation of Eq. 1 on edge-padded images; the
windowed matcher equals the global brute-force matcher when the window covers
the grid, has the closed form of a single candidate at radius 0, and equals a
numpy brute force over each window (ties to the lowest raster index)."""
import numpy as np
import pytest

import oracle
from paper_1609_03986_amd import synth


def numpy_dense(img, x0, y0, gw, gh, triplets):
    """Eq. 1 at every pixel via box sums of G = (C1 - C2)(C1 + C2 - 2A) on the
    edge-padded image: S1 - S2 = sum over the 7 x 7 patch of G."""
    pad = 80
    P = np.pad(img.astype(np.int64), pad, mode="edge")
    out = np.zeros((gh * gw, 16), np.uint32)
    ys, xs = np.mgrid[y0:y0 + gh, x0:x0 + gw]
    for t, tr in enumerate(np.asarray(triplets).reshape(512, 3, 2).astype(np.int64)):
        acc = np.zeros((gh, gw), np.int64)
        for dr in range(-3, 4):
            for dc in range(-3, 4):
                def px(r, c):
                    return P[pad + ys + (r - 24) + dr, pad + xs + (c - 24) + dc]
                a, c1, c2 = px(*tr[0]), px(*tr[1]), px(*tr[2])
                acc += (c1 - c2) * (c1 + c2 - 2 * a)
        bit = (acc > 0).reshape(-1)
        out[:, t // 32] |= (bit.astype(np.uint32) << np.uint32(t % 32))
    return out


def test_dense_equals_box_filter_formulation(triplets):
    g = np.random.default_rng(31)
    img = synth.smoothed_noise(g, 40, 50)
    want = numpy_dense(img, -3, 5, 12, 9, triplets)        # a region crossing the left edge
    got = oracle.extract_dense(img, -3, 5, 12, 9, triplets)
    assert np.array_equal(got, want)


def test_dense_is_extraction_at_the_grid(triplets):
    g = np.random.default_rng(32)
    img = synth.smoothed_noise(g, 60, 70)
    d = oracle.extract_dense(img, 10, 20, 5, 4, triplets)
    for i, (y, x) in enumerate([(yy, xx) for yy in range(20, 24) for xx in range(10, 15)]):
        one, _ = oracle.extract(img, np.array([[x, y, 0, 1]], np.float32), triplets)
        assert np.array_equal(d[i], one[0])


def test_window_covering_the_grid_is_global_knn():
    g = np.random.default_rng(33)
    gw, gh = 9, 7
    q = synth.random_descriptors(g, gw * gh, 0.2)
    t = synth.random_descriptors(g, gw * gh, 0.2)
    t[10] = t[40]                                          # a tie
    wi, wd, wa = oracle.knn_window(q, t, gw, gh, max(gw, gh))
    gi, gd, ga = oracle.knn(q, t)
    assert np.array_equal(wi, gi) and np.array_equal(wd, gd) and np.array_equal(wa, ga)


def test_radius_zero_single_candidate():
    g = np.random.default_rng(34)
    gw, gh = 6, 5
    q = synth.random_descriptors(g, gw * gh)
    t = synth.random_descriptors(g, gw * gh)
    idx, dist, acc = oracle.knn_window(q, t, gw, gh, 0)
    for i in range(gw * gh):
        assert idx[i, 0] == i and dist[i, 0] == oracle.hamming(q[i], t[i])
        assert idx[i, 1] == -1 and dist[i, 1] == 513 and acc[i] == 0


@pytest.mark.parametrize("radius", [1, 2, 3])
def test_window_equals_numpy_brute_force(radius):
    g = np.random.default_rng(35 + radius)
    gw, gh = 8, 6
    q = synth.random_descriptors(g, gw * gh, 0.05)           # many ties
    t = synth.random_descriptors(g, gw * gh, 0.05)
    bits = lambda d: np.unpackbits(d.view(np.uint8), axis=-1).sum(-1)
    idx, dist, acc = oracle.knn_window(q, t, gw, gh, radius, 2, 0.8)
    for y in range(gh):
        for x in range(gw):
            cand = [yy * gw + xx for yy in range(max(0, y - radius), min(gh, y + radius + 1))
                    for xx in range(max(0, x - radius), min(gw, x + radius + 1))]
            d = bits(np.bitwise_xor(q[y * gw + x][None, :], t[cand]))
            order = sorted(range(len(cand)), key=lambda i: (d[i], cand[i]))
            i = y * gw + x
            assert idx[i, 0] == cand[order[0]] and dist[i, 0] == d[order[0]]
            assert idx[i, 1] == cand[order[1]] and dist[i, 1] == d[order[1]]
            # The ratio is a float32 0.8, compared in double.
            assert acc[i] == (d[order[0]] < np.float64(np.float32(0.8)) * d[order[1]])
