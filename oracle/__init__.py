"""LATCH oracle: ctypes wrapper over the plain C implementation in latch_oracle.c.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path
(the HIP library and its Python binding) never imports, links or calls it.

Functions take and return numpy arrays.  See latch_oracle.c for the rule each
function follows and the passage of the paper it implements.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "latch_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

WINDOW = 48
TRIPLETS = 512
WORDS = 16
BINS = 4096
NO_NEIGHBOUR_DIST = 513
FLAG_BAD_KEYPOINT = 1


def build(force=False):
    """Compile latch_oracle.c into liboracle.so with gcc (OpenMP, -O2)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-D_GNU_SOURCE", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        i32 = ctypes.c_int
        lib.oracle_rotation_table.argtypes = [P, P]
        lib.oracle_rotation_table.restype = None
        lib.oracle_sample_window.argtypes = [P, i32, i32, i32, ctypes.c_float, ctypes.c_float,
                                             ctypes.c_float, ctypes.c_float, P, P, P]
        lib.oracle_sample_window.restype = ctypes.c_uint
        lib.oracle_triplet_distances.argtypes = [P, P, P, P]
        lib.oracle_triplet_distances.restype = None
        lib.oracle_describe_tile.argtypes = [P, P, P]
        lib.oracle_describe_tile.restype = None
        lib.oracle_triplets_valid.argtypes = [P]
        lib.oracle_triplets_valid.restype = i32
        lib.oracle_extract.argtypes = [P, i32, i32, i32, P, i64, P, P]
        lib.oracle_extract.restype = ctypes.c_uint
        lib.oracle_hamming.argtypes = [P, P]
        lib.oracle_hamming.restype = i32
        lib.oracle_knn.argtypes = [P, i64, P, i64, i32, ctypes.c_float, P, P, P]
        lib.oracle_knn.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = i32
        lib.oracle_fast_score.argtypes = [P, i32, i32, i32]
        lib.oracle_fast_score.restype = i32
        lib.oracle_orientation_bin.argtypes = [P, i32, i32, i32, P, P]
        lib.oracle_orientation_bin.restype = i32
        lib.oracle_detect.argtypes = [P, i32, i32, i32, i32, P, i64]
        lib.oracle_detect.restype = i64
        lib.oracle_set_threads.argtypes = [i32]
        lib.oracle_set_threads.restype = None
        lib.oracle_sample_window_geom.argtypes = [P, i32, i32, i32, ctypes.c_float, ctypes.c_float,
                                                  ctypes.c_float, ctypes.c_float, P, P, i32, P]
        lib.oracle_sample_window_geom.restype = ctypes.c_uint
        lib.oracle_triplet_distances_weighted.argtypes = [P, i32, i32, P, P, P, P]
        lib.oracle_triplet_distances_weighted.restype = None
        lib.oracle_triplets_valid_geom.argtypes = [P, i32, i32]
        lib.oracle_triplets_valid_geom.restype = i32
        lib.oracle_extract_geom.argtypes = [P, i32, i32, i32, P, i64, P, i32, i32, P, P]
        lib.oracle_extract_geom.restype = ctypes.c_uint
        lib.oracle_knn_window.argtypes = [P, P, i32, i32, i32, i32, ctypes.c_float, P, P, P]
        lib.oracle_knn_window.restype = None
        _lib = lib
    return _lib


def num_threads():
    """OpenMP threads used by extract() and knn()."""
    return int(_load().oracle_num_threads())


DETECT_BORDER = 16
ORIENT_RADIUS = 15


def fast_score(img, x, y):
    """FAST-9 score of pixel (x, y) (the circle must lie inside the image)."""
    img = _image(img)
    return int(_load().oracle_fast_score(_ptr(img), img.shape[1], int(x), int(y)))


def orientation_bin(img, x, y):
    """(bin, m10, m01): intensity-centroid orientation of pixel (x, y)."""
    img = _image(img)
    m10, m01 = ctypes.c_int64(), ctypes.c_int64()
    b = _load().oracle_orientation_bin(_ptr(img), img.shape[1], int(x), int(y),
                                       ctypes.byref(m10), ctypes.byref(m01))
    return int(b), m10.value, m01.value


def detect(img, threshold, max_kps=1 << 20):
    """FAST-9 corners with suppression and orientation: (float32[n, 4] keypoints
    in raster order, total count found)."""
    img = _image(img)
    kps = np.zeros((max_kps, 4), np.float32)
    n = _load().oracle_detect(_ptr(img), img.shape[0], img.shape[1], img.shape[1], int(threshold),
                              _ptr(kps), max_kps)
    if n < 0:
        raise MemoryError("oracle_detect")
    return kps[:min(n, max_kps)].copy(), int(n)


def set_threads(n):
    """Set the OpenMP thread count of extract() and knn() (n >= 1)."""
    _load().oracle_set_threads(int(n))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def rotation_table():
    """Rule R step 2: (cos_q14, sin_q14), two int16 arrays of 4096 bins."""
    c = np.zeros(BINS, np.int16)
    s = np.zeros(BINS, np.int16)
    _load().oracle_rotation_table(_ptr(c), _ptr(s))
    return c, s


def _image(img):
    img = np.ascontiguousarray(img, dtype=np.uint8)
    assert img.ndim == 2
    return img


def sample_window(img, x, y, angle_deg=0.0, scale=1.0):
    """Rule R steps 1-5 for one keypoint: (48x48 uint8 tile, flag)."""
    img = _image(img)
    c, s = rotation_table()
    tile = np.zeros((WINDOW, WINDOW), np.uint8)
    f = _load().oracle_sample_window(_ptr(img), img.shape[0], img.shape[1], img.shape[1],
                                     float(x), float(y), float(angle_deg), float(scale),
                                     _ptr(c), _ptr(s), _ptr(tile))
    return tile, int(f)


def triplet_distances(tile, triplet):
    """Eq. 1 distances (S1, S2) of one triplet {rA, cA, r1, c1, r2, c2} on a tile."""
    tile = np.ascontiguousarray(tile, dtype=np.uint8)
    assert tile.shape == (WINDOW, WINDOW)
    trip = np.ascontiguousarray(np.asarray(triplet, np.uint8).reshape(6))
    s1 = ctypes.c_int64()
    s2 = ctypes.c_int64()
    _load().oracle_triplet_distances(_ptr(tile), _ptr(trip), ctypes.byref(s1), ctypes.byref(s2))
    return s1.value, s2.value


def describe_tile(tile, triplets):
    """Eq. 1 over all 512 triplets of one tile: uint32[16]."""
    tile = np.ascontiguousarray(tile, dtype=np.uint8)
    trip = _triplets(triplets)
    d = np.zeros(WORDS, np.uint32)
    _load().oracle_describe_tile(_ptr(tile), _ptr(trip), _ptr(d))
    return d


def _triplets(triplets):
    trip = np.ascontiguousarray(np.asarray(triplets, np.uint8).reshape(TRIPLETS, 3, 2))
    if not _load().oracle_triplets_valid(_ptr(trip)):
        raise ValueError("triplet centres must lie in [3, 44]")
    return trip


def _keypoints(kps):
    kps = np.ascontiguousarray(np.asarray(kps, np.float32).reshape(-1, 4))
    return kps


def extract(img, kps, triplets):
    """Descriptors uint32[n, 16] and the OR of per-keypoint flags."""
    img = _image(img)
    kps = _keypoints(kps)
    trip = _triplets(triplets)
    n = kps.shape[0]
    desc = np.zeros((n, WORDS), np.uint32)
    f = _load().oracle_extract(_ptr(img), img.shape[0], img.shape[1], img.shape[1],
                               _ptr(kps), n, _ptr(trip), _ptr(desc))
    return desc, int(f)


def _weights(weights, patch):
    if weights is None:
        return np.ones((patch, patch), np.uint8)
    w = np.ascontiguousarray(np.asarray(weights, np.uint8).reshape(patch, patch))
    return w


def sample_window_geom(img, x, y, angle_deg=0.0, scale=1.0, window=64):
    """Rule R with a window of side `window`: (uint8 tile, flag)."""
    img = _image(img)
    c, s = rotation_table()
    tile = np.zeros((window, window), np.uint8)
    f = _load().oracle_sample_window_geom(_ptr(img), img.shape[0], img.shape[1], img.shape[1],
                                          float(x), float(y), float(angle_deg), float(scale),
                                          _ptr(c), _ptr(s), int(window), _ptr(tile))
    return tile, int(f)


def triplet_distances_weighted(tile, triplet, patch=8, weights=None):
    """Weighted distances (S1, S2) of one triplet on a square tile (Sec. 3.2)."""
    tile = np.ascontiguousarray(tile, dtype=np.uint8)
    win = tile.shape[0]
    trip = np.ascontiguousarray(np.asarray(triplet, np.uint8).reshape(6))
    w = _weights(weights, patch)
    s1 = ctypes.c_int64()
    s2 = ctypes.c_int64()
    _load().oracle_triplet_distances_weighted(_ptr(tile), win, int(patch), _ptr(w), _ptr(trip),
                                              ctypes.byref(s1), ctypes.byref(s2))
    return s1.value, s2.value


def triplets_valid_geom(triplets, window, patch):
    trip = np.ascontiguousarray(np.asarray(triplets, np.uint8).reshape(TRIPLETS, 3, 2))
    return bool(_load().oracle_triplets_valid_geom(_ptr(trip), int(window), int(patch)))


def extract_geom(img, kps, triplets, window=64, patch=8, weights=None):
    """Descriptors with window side `window`, patch side `patch` and integer
    weights[patch][patch] (None: all ones), and the OR of the flags."""
    img = _image(img)
    kps = _keypoints(kps)
    trip = np.ascontiguousarray(np.asarray(triplets, np.uint8).reshape(TRIPLETS, 3, 2))
    if not _load().oracle_triplets_valid_geom(_ptr(trip), int(window), int(patch)):
        raise ValueError("every patch must lie inside the window")
    w = _weights(weights, patch)
    n = kps.shape[0]
    desc = np.zeros((n, WORDS), np.uint32)
    f = _load().oracle_extract_geom(_ptr(img), img.shape[0], img.shape[1], img.shape[1], _ptr(kps), n,
                                    _ptr(trip), int(window), int(patch), _ptr(w), _ptr(desc))
    return desc, int(f)


def dense_keypoints(x0, y0, gw, gh):
    """Keypoints (x, y, 0, 1) at every pixel of [x0, x0 + gw) x [y0, y0 + gh), raster order."""
    ys, xs = np.mgrid[y0:y0 + gh, x0:x0 + gw]
    kps = np.zeros((gh * gw, 4), np.float32)
    kps[:, 0] = xs.reshape(-1)
    kps[:, 1] = ys.reshape(-1)
    kps[:, 3] = 1.0
    return kps


def extract_dense(img, x0, y0, gw, gh, triplets):
    """Dense CLATCH (Sec. 6): the descriptor of every pixel of the region,
    upright and at scale 1 -- by definition extraction at those keypoints.
    Returns uint32 [gh * gw, 16] in raster order."""
    desc, _ = extract(img, dense_keypoints(x0, y0, gw, gh), triplets)
    return desc


def knn_window(query, train, gw, gh, radius, k=2, ratio=0.8):
    """Dense matching of two gh x gw descriptor grids: per query pixel the k
    nearest train pixels within +/- radius rows and columns (raster indices)."""
    q = np.ascontiguousarray(np.asarray(query, np.uint32).reshape(gh * gw, WORDS))
    t = np.ascontiguousarray(np.asarray(train, np.uint32).reshape(gh * gw, WORDS))
    n = gh * gw
    idx = np.zeros((n, k), np.int32)
    dist = np.zeros((n, k), np.int32)
    acc = np.zeros(n, np.uint8)
    _load().oracle_knn_window(_ptr(q), _ptr(t), int(gw), int(gh), int(radius), int(k), float(ratio),
                              _ptr(idx), _ptr(dist), _ptr(acc))
    return idx, dist, acc


def hamming(a, b):
    a = np.ascontiguousarray(a, np.uint32).reshape(WORDS)
    b = np.ascontiguousarray(b, np.uint32).reshape(WORDS)
    return int(_load().oracle_hamming(_ptr(a), _ptr(b)))


def knn(query, train, k=2, ratio=0.8):
    """Brute-force k-NN: (idx int32[nq,k], dist int32[nq,k], accept uint8[nq])."""
    if k not in (1, 2):
        raise ValueError("k must be 1 or 2")
    q = np.ascontiguousarray(np.asarray(query, np.uint32).reshape(-1, WORDS))
    t = np.ascontiguousarray(np.asarray(train, np.uint32).reshape(-1, WORDS))
    nq, nt = q.shape[0], t.shape[0]
    idx = np.zeros((nq, k), np.int32)
    dist = np.zeros((nq, k), np.int32)
    acc = np.zeros(nq, np.uint8)
    _load().oracle_knn(_ptr(q), nq, _ptr(t), nt, k, float(np.float32(ratio)),
                       _ptr(idx), _ptr(dist), _ptr(acc))
    return idx, dist, acc
