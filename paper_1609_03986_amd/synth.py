"""Seeded synthetic inputs for the LATCH extraction + matching path.

This module only draws inputs: images, keypoints, triplet tables and the
shifted-plus-noise twin of an image.  It holds none of the method's
arithmetic (no sampling rule, no patch distances, no Hamming distances), so
that both the HIP path and the CPU oracle can be driven from it.

Seeds: numpy PCG64 with seed = 160903986 + 1000 * workload + stream, where the
streams are 0 image, 1 keypoints, 2 noise/shift, 3 arrivals; the triplet table
uses seed 160903986 with stream 9 and is shared by every workload.

Workloads (stand-ins for the paper's Strecha et al. photogrammetry scenes,
5616 x 3744 images, Sec. 5, which are not available):
  1 "small":  640x480 smoothed noise, 2,000 upright keypoints on a jittered grid.
  2 "hd":     1920x1080 smoothed noise + rectangles + blobs, 10,000 keypoints with
              angle U[0, 360) and scale 1.2^L, L ~ U{0..7}.
  3 "sfm":    64 crops of 3000x2000 from one textured mosaic (offsets 16 px / 8 px,
              +-4 noise), 20,000 keypoints each as in "hd"; the 63 consecutive
              image pairs are matched.
  4 "uneven": 256 images, sizes uniform over {320x240, 640x480, 1280x720,
              1920x1080, 4000x3000}, keypoints per image round(LogNormal(ln 5000, 1))
              clipped to [500, 50000]; the 255 consecutive pairs are matched.
"""
import numpy as np
from scipy.ndimage import gaussian_filter

BASE_SEED = 160903986
WINDOW = 48
TRIPLET_LO, TRIPLET_HI = 3, 44       # patch centres keep the 7x7 patch inside the window
TRIPLETS = 512

STREAM_IMAGE, STREAM_KEYPOINTS, STREAM_NOISE, STREAM_ARRIVALS = 0, 1, 2, 3


def rng(workload, stream):
    return np.random.Generator(np.random.PCG64(BASE_SEED + 1000 * workload + stream))


def triplet_table(seed_stream=9):
    """512 triplets {(rA, cA), (r1, c1), (r2, c2)}, centres uniform in [3, 44].

    The learned table of the paper (trained on Brown et al. patches, Sec. 3.1)
    is not available; seeded uniform triplets stand in for it.  Triplets with
    two equal centres are redrawn so that every bit carries information.
    Returns uint8 [512, 3, 2].
    """
    g = np.random.Generator(np.random.PCG64(BASE_SEED + seed_stream))
    out = np.zeros((TRIPLETS, 3, 2), np.uint8)
    t = 0
    while t < TRIPLETS:
        c = g.integers(TRIPLET_LO, TRIPLET_HI + 1, size=(3, 2))
        a, p, q = (tuple(r) for r in c)
        if a == p or a == q or p == q:
            continue
        out[t] = c
        t += 1
    return out


def triplet_table_geom(window=64, patch=8, seed_stream=10):
    """512 triplets for a window of side `window` and patches of side `patch`:
    centres uniform over the positions whose patch (top-left at centre -
    patch // 2) lies inside the window, i.e. [patch // 2, window - patch + patch // 2].
    Seeded uniform triplets stand in for the learned table; triplets with two
    equal centres are redrawn.  Returns uint8 [512, 3, 2]."""
    lo, hi = patch // 2, window - patch + patch // 2
    g = np.random.Generator(np.random.PCG64(BASE_SEED + seed_stream))
    out = np.zeros((TRIPLETS, 3, 2), np.uint8)
    t = 0
    while t < TRIPLETS:
        c = g.integers(lo, hi + 1, size=(3, 2))
        a, p, q = (tuple(r) for r in c)
        if a == p or a == q or p == q:
            continue
        out[t] = c
        t += 1
    return out


def gaussian_weights(patch=8, sigma=2.0, peak=128):
    """Integer weights[patch][patch]: peak * exp(-r^2 / (2 sigma^2)) rounded,
    r the distance from the patch centre ((patch - 1) / 2 in each axis)."""
    c = (patch - 1) / 2.0
    i = np.arange(patch, dtype=np.float64) - c
    r2 = i[:, None] ** 2 + i[None, :] ** 2
    return np.rint(peak * np.exp(-r2 / (2.0 * sigma * sigma))).astype(np.uint8)


def clatch_7x7_weights():
    """8 x 8 weights emulating the 7 x 7 patch (Sec. 3.2): zero on the first
    row and the first column, one elsewhere."""
    w = np.ones((8, 8), np.uint8)
    w[0, :] = 0
    w[:, 0] = 0
    return w


def smoothed_noise(g, height, width, sigma=1.5, mean=128.0, std=48.0):
    """i.i.d. U{0..255}, Gaussian sigma (radius 5, reflect), stretched to mean/std."""
    raw = g.integers(0, 256, size=(height, width)).astype(np.float64)
    sm = gaussian_filter(raw, sigma, mode="reflect", truncate=5.0 / sigma)
    sm = (sm - sm.mean()) / max(sm.std(), 1e-9) * std + mean
    return np.clip(np.rint(sm), 0, 255).astype(np.uint8)


def textured_image(g, height, width, n_rect=200, n_blob=200):
    """Smoothed noise plus random filled rectangles and Gaussian blobs."""
    img = smoothed_noise(g, height, width).astype(np.float64)
    for _ in range(n_rect):
        h, w = g.integers(8, 201, size=2)
        y0 = g.integers(0, max(1, height - h))
        x0 = g.integers(0, max(1, width - w))
        level = g.integers(0, 256)
        img[y0:y0 + h, x0:x0 + w] = 0.5 * img[y0:y0 + h, x0:x0 + w] + 0.5 * level
    for _ in range(n_blob):
        sig = g.uniform(3.0, 30.0)
        amp = g.uniform(-80.0, 80.0)
        cy, cx = g.uniform(0, height), g.uniform(0, width)
        r = int(3 * sig) + 1
        y0, y1 = max(0, int(cy) - r), min(height, int(cy) + r + 1)
        x0, x1 = max(0, int(cx) - r), min(width, int(cx) + r + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        yy, xx = np.mgrid[y0:y1, x0:x1]
        img[y0:y1, x0:x1] += amp * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * sig * sig))
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def shifted_twin(g, img, dx=3, dy=2, noise=4):
    """I2[y][x] = clip(I1[y - dy][x - dx] + U{-noise..noise}), source index clamped."""
    h, w = img.shape
    ys = np.clip(np.arange(h) - dy, 0, h - 1)
    xs = np.clip(np.arange(w) - dx, 0, w - 1)
    src = img[ys][:, xs].astype(np.int32)
    if noise:
        src = src + g.integers(-noise, noise + 1, size=src.shape)
    return np.clip(src, 0, 255).astype(np.uint8)


def grid_keypoints(g, nx, ny, x0, x1, y0, y1, jitter=0.45):
    """nx * ny upright keypoints on a jittered grid over [x0, x1) x [y0, y1)."""
    cw, ch = (x1 - x0) / nx, (y1 - y0) / ny
    gx, gy = np.meshgrid(np.arange(nx), np.arange(ny))
    x = x0 + (gx.ravel() + 0.5) * cw + g.uniform(-jitter, jitter, nx * ny) * cw
    y = y0 + (gy.ravel() + 0.5) * ch + g.uniform(-jitter, jitter, nx * ny) * ch
    kps = np.zeros((nx * ny, 4), np.float32)
    kps[:, 0] = x
    kps[:, 1] = y
    kps[:, 3] = 1.0
    return kps


def random_keypoints(g, n, height, width, margin=16, levels=8, factor=1.2):
    """n keypoints uniform in [margin, W - margin) x [margin, H - margin),
    angle U[0, 360) degrees, scale factor^L with L ~ U{0..levels-1}."""
    kps = np.zeros((n, 4), np.float32)
    kps[:, 0] = g.uniform(margin, width - margin, n)
    kps[:, 1] = g.uniform(margin, height - margin, n)
    kps[:, 2] = g.uniform(0.0, 360.0, n)
    kps[:, 3] = factor ** g.integers(0, levels, n)
    return kps


def workload_small():
    """One 640x480 image, 2,000 upright keypoints, and its shifted (3, 2) +/-4 twin."""
    img = smoothed_noise(rng(1, STREAM_IMAGE), 480, 640)
    kps = grid_keypoints(rng(1, STREAM_KEYPOINTS), 50, 40, 32, 608, 32, 448)
    twin = shifted_twin(rng(1, STREAM_NOISE), img)
    kps2 = kps.copy()
    kps2[:, 0] += 3
    kps2[:, 1] += 2
    return dict(name="640x480, 2,000 upright keypoints", query_image=img, query_kps=kps,
                train_image=twin, train_kps=kps2)


def workload_hd(n_kps=10000):
    """One 1920x1080 textured image, 10,000 oriented and scaled keypoints, and its twin."""
    img = textured_image(rng(2, STREAM_IMAGE), 1080, 1920)
    kps = random_keypoints(rng(2, STREAM_KEYPOINTS), n_kps, 1080, 1920)
    twin = shifted_twin(rng(2, STREAM_NOISE), img)
    kps2 = kps.copy()
    kps2[:, 0] += 3
    kps2[:, 1] += 2
    return dict(name="1920x1080, %d keypoints, random angle and scale" % n_kps,
                query_image=img, query_kps=kps, train_image=twin, train_kps=kps2)


def random_descriptors(g, n, p_one=0.5):
    """n random 512-bit descriptors as uint32[n, 16] (bits i.i.d. Bernoulli(p_one))."""
    bits = (g.random((n, 512)) < p_one).astype(np.uint8)
    return np.packbits(bits, axis=1, bitorder="little").view(np.uint32).reshape(n, 16)


UNEVEN_SIZES = [(240, 320), (480, 640), (720, 1280), (1080, 1920), (3000, 4000)]


def sfm_workload(n_img=64, h=2000, w=3000, n_kp=20000, seed=BASE_SEED + 3000):
    """Workload 3: n_img crops of h x w from one textured mosaic of
    (h + 8 (n_img - 1)) x (w + 16 (n_img - 1)), crop i at (16 i, 8 i) plus
    U{-4..4} noise, and n_kp random keypoints per image.  Returns (images, keypoints)."""
    g = np.random.default_rng(seed)
    mosaic = textured_image(g, h + 8 * (n_img - 1), w + 16 * (n_img - 1))
    imgs = []
    for i in range(n_img):
        crop = mosaic[8 * i:8 * i + h, 16 * i:16 * i + w].astype(np.int16)
        imgs.append(np.clip(crop + g.integers(-4, 5, crop.shape, dtype=np.int16), 0, 255)
                    .astype(np.uint8))
    kps = [random_keypoints(g, n_kp, h, w) for _ in range(n_img)]
    return imgs, kps


def uneven_workload(n_img=256, seed=BASE_SEED + 4000, pool_per_size=2):
    """Workload 4: image sizes uniform over UNEVEN_SIZES, keypoint counts
    round(LogNormal(ln 5000, 1)) clipped to [500, 50000].  Pixel data comes
    from a small seeded pool per size (copied into distinct device buffers by
    the caller); keypoints are drawn per image.  Returns (images, keypoints)."""
    g = np.random.default_rng(seed)
    pool = {hw: [smoothed_noise(g, *hw) for _ in range(pool_per_size)] for hw in UNEVEN_SIZES}
    imgs, kps = [], []
    for _ in range(n_img):
        hw = UNEVEN_SIZES[int(g.integers(0, len(UNEVEN_SIZES)))]
        imgs.append(pool[hw][int(g.integers(0, pool_per_size))])
        n = int(np.clip(np.rint(g.lognormal(np.log(5000), 1.0)), 500, 50000))
        kps.append(random_keypoints(g, n, *hw))
    return imgs, kps
