"""GPU parity of dense CLATCH (latch_extract_dense) and dense windowed matching
(hamming_knn_window), Sec. 6: descriptors bit-exactly equal to the oracle's
extraction at every pixel (regions crossing the image edges, ragged tiles,
single rows and columns), equal to the sparse path at the same keypoints, and
windowed 2-NN equal to the oracle for every radius class."""
import numpy as np
import pytest

import oracle
from paper_1609_03986_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def lat(torch_cuda, triplets):
    from paper_1609_03986_amd.binding import Latch
    L = Latch(triplets)
    yield L
    L.close()


def u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("region", [(-5, -7, 75, 40), (0, 0, 90, 70), (60, 30, 58, 32), (20, 10, 1, 33),
                                    (3, 44, 117, 1), (85, 65, 12, 9)])
def test_dense_matches_oracle(torch_cuda, lat, triplets, region):
    g = np.random.default_rng(sum(region) + 1000)
    img = synth.smoothed_noise(g, 70, 90)
    x0, y0, gw, gh = region
    d = lat.extract_dense(torch_cuda.from_numpy(img).cuda(), x0, y0, gw, gh)
    torch_cuda.cuda.synchronize()
    want = oracle.extract_dense(img, x0, y0, gw, gh, triplets)
    bad = np.nonzero((u32(d) != want).any(1))[0]
    assert bad.size == 0, (region, bad[:10])


def test_dense_equals_sparse_path(torch_cuda, lat):
    torch = torch_cuda
    g = np.random.default_rng(41)
    img = torch.from_numpy(synth.textured_image(g, 240, 320, n_rect=40, n_blob=40)).cuda()
    x0, y0, gw, gh = 17, 9, 203, 150
    d = lat.extract_dense(img, x0, y0, gw, gh)
    kps = torch.from_numpy(oracle.dense_keypoints(x0, y0, gw, gh)).cuda()
    s = lat.extract(img, kps)
    torch.cuda.synchronize()
    assert torch.equal(d, s)


def test_dense_hd_sampled(torch_cuda, lat, triplets):
    """Every pixel of the 1920 x 1080 bench image in one launch; every 997th
    descriptor against the oracle."""
    torch = torch_cuda
    img = synth.workload_hd()["query_image"]
    H, W = img.shape
    d = u32(lat.extract_dense(torch.from_numpy(img).cuda(), 0, 0, W, H))
    sel = np.arange(0, H * W, 997)
    kps = oracle.dense_keypoints(0, 0, W, H)[sel]
    want, _ = oracle.extract(img, kps, triplets)
    assert np.array_equal(d[sel], want)


@pytest.mark.parametrize("radius", [0, 1, 3, 8])
@pytest.mark.parametrize("k", [1, 2])
def test_window_matching_matches_oracle(torch_cuda, lat, radius, k):
    torch = torch_cuda
    g = np.random.default_rng(50 + radius)
    gw, gh = 37, 29                                      # ragged against 16 x 16 tiles
    q = synth.random_descriptors(g, gw * gh, 0.05)        # tie-heavy
    t = synth.random_descriptors(g, gw * gh, 0.05)
    t[100:140] = q[100:140]                               # exact matches
    qd = torch.from_numpy(q.view(np.int32)).cuda()
    td = torch.from_numpy(t.view(np.int32)).cuda()
    idx, dist, acc = lat.knn_window(qd, td, gw, gh, radius, k=k, ratio=0.8)
    torch.cuda.synchronize()
    wi, wd, wa = oracle.knn_window(q, t, gw, gh, radius, k, 0.8)
    assert np.array_equal(idx.cpu().numpy(), wi)
    assert np.array_equal(dist.cpu().numpy(), wd)
    assert np.array_equal(acc.cpu().numpy(), wa)


def test_dense_flow_of_a_shifted_twin(torch_cuda, lat, triplets):
    """Dense descriptors of an image and its copy shifted by (3, 2) with noise,
    matched within radius 4: oracle parity on a sample, and most accepted
    matches recover the shift."""
    torch = torch_cuda
    g = np.random.default_rng(60)
    img = synth.textured_image(g, 120, 160, n_rect=30, n_blob=30)
    twin = np.clip(np.roll(img, (2, 3), axis=(0, 1)).astype(int) + g.integers(-4, 5, img.shape), 0, 255).astype(np.uint8)
    gw, gh = 160, 120
    a = lat.extract_dense(torch.from_numpy(img).cuda(), 0, 0, gw, gh)
    b = lat.extract_dense(torch.from_numpy(twin).cuda(), 0, 0, gw, gh)
    idx, dist, acc = lat.knn_window(a, b, gw, gh, 4)
    torch.cuda.synchronize()
    A, B = u32(a), u32(b)
    wi, wd, wa = oracle.knn_window(A, B, gw, gh, 4)
    assert np.array_equal(idx.cpu().numpy(), wi) and np.array_equal(acc.cpu().numpy(), wa)
    i = np.arange(gw * gh)
    inner = ((i // gw) >= 30) & ((i // gw) < gh - 30) & ((i % gw) >= 30) & ((i % gw) < gw - 30)
    ok = acc.cpu().numpy().astype(bool) & inner
    found = idx.cpu().numpy()[:, 0]
    assert ok.sum() > 1000
    assert np.mean(found[ok] == i[ok] + 2 * gw + 3) > 0.9


def test_bad_arguments(torch_cuda, lat, triplets):
    from paper_1609_03986_amd.binding import LATCH_EINVAL, LATCH_ERANGE, Latch, LatchError
    torch = torch_cuda
    d = torch.zeros((16, 16), dtype=torch.int32, device="cuda")
    with pytest.raises(LatchError) as e:
        lat.knn_window(d, d, 4, 4, 9)
    assert e.value.code == LATCH_ERANGE
    geo = Latch(synth.triplet_table_geom(64, 8), 64, 8)
    try:
        with pytest.raises(LatchError) as e:
            geo.extract_dense(torch.zeros((64, 64), dtype=torch.uint8, device="cuda"), 0, 0, 4, 4)
        assert e.value.code == LATCH_EINVAL
    finally:
        geo.close()
    with pytest.raises(LatchError) as e:
        lat.extract_dense(torch.zeros((64, 64), dtype=torch.uint8, device="cuda"), 1 << 24, 0, 4, 4)
    assert e.value.code == LATCH_ERANGE
