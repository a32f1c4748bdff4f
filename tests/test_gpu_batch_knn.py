"""GPU parity of batched matching (hamming_knn_batch): many query/train pairs
in one persistent launch, each pair exactly equal to the oracle's brute-force
2-NN on its ranges and to the single hamming_knn call."""
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
    L.check_errors(clear=True)
    yield L
    L.close()


def dev(torch, d):
    return torch.from_numpy(np.ascontiguousarray(d, np.uint32).view(np.int32)).cuda()


def consecutive_pairs(counts):
    """Pairs (i, i + 1) of images with `counts` descriptors each, in one array."""
    first = np.concatenate([[0], np.cumsum(counts)[:-1]])
    rows, out = [], 0
    for i in range(len(counts) - 1):
        rows.append((first[i], counts[i], first[i + 1], counts[i + 1], out))
        out += counts[i]
    return rows, out


def check_pairs(torch, lat, D, rows, out_rows, k, ratio, path):
    from paper_1609_03986_amd.binding import pair_table
    Dd = dev(torch, D)
    idx, dist, acc = lat.knn_batch(Dd, Dd, pair_table(rows), out_rows, k=k, ratio=ratio, path=path)
    torch.cuda.synchronize()
    idx, dist, acc = idx.cpu().numpy(), dist.cpu().numpy(), acc.cpu().numpy()
    for qf, nq, tf, nt, of in rows:
        wi, wd, wa = oracle.knn(D[qf:qf + nq], D[tf:tf + nt], k=k, ratio=ratio)
        assert np.array_equal(idx[of:of + nq], wi), (path, qf, nq, tf, nt)
        assert np.array_equal(dist[of:of + nq], wd), (path, qf, nq, tf, nt)
        assert np.array_equal(acc[of:of + nq], wa), (path, qf, nq, tf, nt)
    return idx, dist, acc


@pytest.mark.parametrize("path", ["mfma", "fp4", "popcount"])
def test_uneven_consecutive_pairs(torch_cuda, lat, path):
    g = np.random.default_rng(7)
    counts = [300, 0, 257, 1, 2, 511, 33, 1000, 640, 5]
    D = synth.random_descriptors(g, sum(counts), 0.3)
    D[100:140] = D[400:440]                       # cross-image duplicates: ties
    rows, out_rows = consecutive_pairs(counts)
    for k in (1, 2):
        check_pairs(torch_cuda, lat, D, rows, out_rows, k, 0.8, path)
    assert lat.check_errors(clear=True) == 0


def test_batch_equals_single_calls(torch_cuda, lat):
    g = np.random.default_rng(8)
    counts = [700, 900, 650, 1200]
    D = synth.random_descriptors(g, sum(counts))
    rows, out_rows = consecutive_pairs(counts)
    idx, dist, acc = check_pairs(torch_cuda, lat, D, rows, out_rows, 2, 0.8, "auto")
    for qf, nq, tf, nt, of in rows:
        si, sd, sa = lat.knn(dev(torch_cuda, D[qf:qf + nq]), dev(torch_cuda, D[tf:tf + nt]))
        torch_cuda.cuda.synchronize()
        assert np.array_equal(si.cpu().numpy(), idx[of:of + nq])
        assert np.array_equal(sd.cpu().numpy(), dist[of:of + nq])
        assert np.array_equal(sa.cpu().numpy(), acc[of:of + nq])


def test_out_of_range_pair_is_flagged_and_skipped(torch_cuda, lat):
    from paper_1609_03986_amd.binding import FLAG_BAD_PAIR, pair_table
    g = np.random.default_rng(9)
    D = synth.random_descriptors(g, 400)
    rows = [(0, 100, 100, 100, 0), (200, 100, 350, 100, 100), (300, 50, 0, 200, 200)]  # 2nd: train past the end
    Dd = dev(torch_cuda, D)
    idx, dist, acc = lat.knn_batch(Dd, Dd, pair_table(rows), 250)
    torch_cuda.cuda.synchronize()
    assert lat.check_errors(clear=True) & FLAG_BAD_PAIR
    idx = idx.cpu().numpy()
    assert np.all(idx[100:200] == -2)             # untouched
    wi, _, _ = oracle.knn(D[0:100], D[100:200])
    assert np.array_equal(idx[0:100], wi)
    wi, _, _ = oracle.knn(D[300:350], D[0:200])
    assert np.array_equal(idx[200:250], wi)


def test_sfm_shaped_batch_sampled(torch_cuda, lat, triplets):
    """Eight overlapping crops of one mosaic, 3,000 keypoints each, extracted in
    one batched launch and matched as 7 consecutive pairs in one batched launch;
    every 9th query of every pair checked against the oracle."""
    from paper_1609_03986_amd.binding import image_table, pair_table
    torch = torch_cuda
    g = np.random.default_rng(64)
    H, W, n_img, n_kp = 600, 800, 8, 3000
    mosaic = synth.textured_image(g, H + 16 * n_img, W + 16 * n_img, n_rect=60, n_blob=60)
    imgs = [np.clip(mosaic[8 * i:8 * i + H, 16 * i:16 * i + W].astype(int)
                    + g.integers(-4, 5, (H, W)), 0, 255).astype(np.uint8) for i in range(n_img)]
    kps = np.concatenate([synth.random_keypoints(g, n_kp, H, W) for _ in range(n_img)])
    ids = np.repeat(np.arange(n_img, dtype=np.int32), n_kp)
    dimgs = [torch.from_numpy(im).cuda() for im in imgs]
    desc = lat.extract_batch(image_table(dimgs), n_img, torch.from_numpy(ids).cuda(),
                             torch.from_numpy(kps).cuda())
    rows, out_rows = consecutive_pairs([n_kp] * n_img)
    idx, dist, acc = lat.knn_batch(desc, desc, pair_table(rows), out_rows)
    torch.cuda.synchronize()
    D = desc.cpu().numpy().view(np.uint32)
    want_d, f = oracle.extract(imgs[3], kps[3 * n_kp:4 * n_kp], triplets)
    assert np.array_equal(D[3 * n_kp:4 * n_kp], want_d)
    idx, dist, acc = idx.cpu().numpy(), dist.cpu().numpy(), acc.cpu().numpy()
    for qf, nq, tf, nt, of in rows:
        sel = np.arange(0, nq, 9)
        wi, wd, wa = oracle.knn(D[qf + sel], D[tf:tf + nt])
        assert np.array_equal(idx[of + sel], wi)
        assert np.array_equal(dist[of + sel], wd)
        assert np.array_equal(acc[of + sel], wa)
    assert lat.check_errors(clear=True) == 0


@pytest.mark.parametrize("path", ["fp4", "mfma"])
def test_long_train_ranges(torch_cuda, lat, path):
    """Pairs whose train range exceeds 2^14 rows: the MXFP4 batch matcher scans
    such a range in pieces of 2^14 rows and merges them in registers; ties
    across piece boundaries resolve to the lowest index."""
    g = np.random.default_rng(12)
    counts = [70, 16385, 300, 40000, 5]
    D = synth.random_descriptors(g, sum(counts), 0.05)
    D[70 + 16384] = D[70]                         # tie across the 2^14 boundary of pair 0
    D[70 + 16385 + 300 + 20000] = D[70 + 16385 + 5]
    rows, out_rows = consecutive_pairs(counts)
    check_pairs(torch_cuda, lat, D, rows, out_rows, 2, 0.8, path)
    assert lat.check_errors(clear=True) == 0


@pytest.mark.parametrize("path", ["fp4", "mfma"])
def test_many_pairs_across_cost_classes(torch_cuda, lat, path):
    """700 pairs (more than the setup block's 256 threads) in random order,
    train lengths log-uniform over 0..20,000 rows (work items laid out over
    several dozen cost classes, longest first), query counts 0..300, train
    ranges overlapping anywhere in the array: every pair's rows equal the
    single hamming_knn call on its ranges, and a sample equals the oracle."""
    from paper_1609_03986_amd.binding import pair_table
    torch = torch_cuda
    g = np.random.default_rng(21)
    n_rows = 30_000
    D = synth.random_descriptors(g, n_rows, 0.2)
    n_pairs = 700
    nt = np.floor(np.exp(g.uniform(0, np.log(20_001), n_pairs))).astype(np.int64) - 1
    nt[g.choice(n_pairs, 20, replace=False)] = 0
    nq = g.integers(0, 301, n_pairs)
    rows, out = [], 0
    for i in range(n_pairs):
        qf = int(g.integers(0, n_rows - nq[i] + 1))
        tf = int(g.integers(0, n_rows - nt[i] + 1))
        rows.append((qf, int(nq[i]), tf, int(nt[i]), out))
        out += int(nq[i])
    Dd = dev(torch, D)
    idx, dist, acc = lat.knn_batch(Dd, Dd, pair_table(rows), out, path=path)
    torch.cuda.synchronize()
    assert lat.check_errors(clear=True) == 0
    idx, dist, acc = idx.cpu().numpy(), dist.cpu().numpy(), acc.cpu().numpy()
    for i, (qf, q, tf, t, of) in enumerate(rows):
        if q == 0:
            continue
        si, sd, sa = lat.knn(Dd[qf:qf + q], Dd[tf:tf + t], path=path)
        torch.cuda.synchronize()
        assert np.array_equal(idx[of:of + q], si.cpu().numpy()), (i, q, t)
        assert np.array_equal(dist[of:of + q], sd.cpu().numpy()), (i, q, t)
        assert np.array_equal(acc[of:of + q], sa.cpu().numpy()), (i, q, t)
        if i % 7 == 0:
            sel = np.arange(0, q, 37)
            wi, wd, wa = oracle.knn(D[qf + sel], D[tf:tf + t])
            assert np.array_equal(idx[of + sel], wi), (i, q, t)
            assert np.array_equal(dist[of + sel], wd), (i, q, t)
            assert np.array_equal(acc[of + sel], wa), (i, q, t)
    assert lat.check_errors(clear=True) == 0
