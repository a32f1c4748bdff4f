"""GPU parity: HIP 2-NN Hamming matching (int8 MFMA, MXFP4 MFMA and popcount paths) through the
C ABI vs the CPU oracle, exact: indices, distances and ratio-test flags.

Covers empty and tiny sets, sizes around the 32-row tile and 256-query group,
many train splits, heavy ties (sparse bits, duplicate rows), all-zero and
all-one descriptors, k = 1 and 2, the ratio-test edges, and the 10k x 10k
workload built from real extracted descriptors.
"""
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


def to_dev(torch, d):
    return torch.from_numpy(np.ascontiguousarray(d, np.uint32).view(np.int32)).cuda()


def gpu_knn(torch, lat, Q, T, k, ratio, path):
    idx, dist, acc = lat.knn(to_dev(torch, Q), to_dev(torch, T.reshape(-1, 16)), k=k, ratio=ratio,
                             path=path)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy(), acc.cpu().numpy()


def check(torch, lat, Q, T, k=2, ratio=0.8, paths=("mfma", "fp4", "popcount")):
    wi, wd, wa = oracle.knn(Q, T, k=k, ratio=ratio)
    for path in paths:
        gi, gd, ga = gpu_knn(torch, lat, Q, T, k, ratio, path)
        for name, g, w in (("idx", gi, wi), ("dist", gd, wd), ("accept", ga, wa)):
            if not np.array_equal(g, w):
                bad = np.nonzero((g != w).reshape(len(Q), -1).any(1))[0]
                raise AssertionError("%s path: %s differs on %d of %d queries, first q=%d: "
                                     "got %s want %s" % (path, name, len(bad), len(Q), bad[0],
                                                         g[bad[0]], w[bad[0]]))


SIZES = [(1, 0), (1, 1), (1, 2), (5, 3), (31, 33), (32, 32), (33, 31), (64, 64), (255, 257),
         (257, 300), (1000, 2000), (2048, 4096), (300, 20000), (3, 70000)]


@pytest.mark.parametrize("nq,nt", SIZES)
def test_random_sets(torch_cuda, lat, nq, nt):
    g = np.random.default_rng(nq * 100003 + nt)
    Q = synth.random_descriptors(g, nq)
    T = synth.random_descriptors(g, nt) if nt else np.zeros((0, 16), np.uint32)
    for k in (1, 2):
        check(torch_cuda, lat, Q, T, k=k)


@pytest.mark.parametrize("p", [0.02, 0.002])
def test_heavy_ties_and_duplicates(torch_cuda, lat, p):
    g = np.random.default_rng(int(p * 1e4))
    Q = synth.random_descriptors(g, 700, p)
    T = synth.random_descriptors(g, 3000, p)
    T[1000:1100] = T[:100]
    T[2999] = T[5]
    Q[:50] = T[900:950]
    check(torch_cuda, lat, Q, T)


def test_all_zero_and_all_one_rows(torch_cuda, lat):
    g = np.random.default_rng(11)
    Q = synth.random_descriptors(g, 100)
    T = synth.random_descriptors(g, 500)
    Q[0] = 0
    Q[1] = 0xFFFFFFFF
    T[7] = 0
    T[400] = 0xFFFFFFFF
    T[401] = 0xFFFFFFFF
    check(torch_cuda, lat, Q, T)
    check(torch_cuda, lat, np.zeros((40, 16), np.uint32), np.zeros((70, 16), np.uint32))
    ones = np.full((40, 16), 0xFFFFFFFF, np.uint32)
    check(torch_cuda, lat, ones, np.concatenate([np.zeros((3, 16), np.uint32), ones]))


@pytest.mark.parametrize("ratio", [0.75, 0.8, 0.999, 1.0, 1e-6])
def test_ratio_values(torch_cuda, lat, ratio):
    g = np.random.default_rng(17)
    Q = synth.random_descriptors(g, 400, 0.05)
    T = synth.random_descriptors(g, 900, 0.05)
    check(torch_cuda, lat, Q, T, ratio=ratio)


def test_ratio_edges_exact(torch_cuda, lat):
    Q = np.zeros((1, 16), np.uint32)
    for d1, d2, ratio in [(4, 5, 0.8), (8, 10, 0.8), (3, 4, 0.75), (0, 0, 0.8), (9, 11, 0.8)]:
        T = np.zeros((3, 16), np.uint32)
        for r, nbits in enumerate([d2, d1, 512]):
            b = np.zeros(512, np.uint8)
            b[:nbits] = 1
            T[r] = np.packbits(b, bitorder="little").view(np.uint32)
        check(torch_cuda, lat, Q, T, ratio=ratio)


def test_hd_workload_full_10k_by_10k(torch_cuda, lat, triplets):
    """The 1920x1080 workload: 10,000 query and 10,000 train descriptors from the
    HIP extractor (checked bit-exact in the extraction tests), matched in full."""
    torch = torch_cuda
    w = synth.workload_hd()
    dq = lat.extract(torch.from_numpy(w["query_image"]).cuda(),
                     torch.from_numpy(w["query_kps"]).cuda())
    dt = lat.extract(torch.from_numpy(w["train_image"]).cuda(),
                     torch.from_numpy(w["train_kps"]).cuda())
    torch.cuda.synchronize()
    Q = dq.cpu().numpy().view(np.uint32)
    T = dt.cpu().numpy().view(np.uint32)
    check(torch, lat, Q, T)
    _, dist, acc = oracle.knn(Q, T)
    assert acc.mean() > 0.3          # sanity: the twin image matches


def test_auto_path_equals_explicit(torch_cuda, lat):
    g = np.random.default_rng(23)
    Q = synth.random_descriptors(g, 500)
    T = synth.random_descriptors(g, 1500)
    check(torch_cuda, lat, Q, T, paths=("auto",))


def test_bad_arguments_raise(torch_cuda, lat):
    from paper_1609_03986_amd.binding import LatchError
    q = to_dev(torch_cuda, np.zeros((4, 16), np.uint32))
    for kw, code in [(dict(k=3), -4), (dict(k=0), -4), (dict(ratio=0.0), -4),
                     (dict(ratio=1.5), -4), (dict(ratio=float("nan")), -4)]:
        args = dict(k=2, ratio=0.8)
        args.update(kw)
        with pytest.raises(LatchError) as e:
            lat.knn(q, q, **args)
        assert e.value.code == code
    idx, dist, acc = lat.knn(q[:0], q)          # nq = 0 is a no-op
    assert idx.shape == (0, 2)


def test_split_merge_repeated_calls(torch_cuda, lat):
    """The split merge's per-group counters return to zero after every call:
    alternating shapes with many train splits on one handle stay exact."""
    g = np.random.default_rng(77)
    shapes = [(600, 50000), (2000, 9000), (600, 50000), (257, 123457), (2000, 9000)]
    for nq, nt in shapes:
        Q = synth.random_descriptors(g, nq)
        T = synth.random_descriptors(g, nt)
        check(torch_cuda, lat, Q, T, k=2)


def test_fp4_split_boundaries(torch_cuda, lat):
    """MXFP4 keys hold a 14-bit split-local index: train sets around and above
    2^14 rows force several splits, with ties across split edges."""
    g = np.random.default_rng(91)
    for nq, nt in [(40, 16384), (40, 16385), (300, 16416), (97, 40000)]:
        Q = synth.random_descriptors(g, nq, p_one=0.02)
        T = synth.random_descriptors(g, nt, p_one=0.02)
        T[-1] = T[0]                                  # an exact tie across the whole set
        check(torch_cuda, lat, Q, T, paths=("fp4", "mfma"))


@pytest.mark.parametrize("path", ["fp4", "mfma"])
@pytest.mark.parametrize("nq,nt", [(20_000, 20_000), (100_000, 100_000)])
def test_split_counts_that_fill_the_last_round(torch_cuda, lat, nq, nt, path):
    """Shapes where the split planner takes more splits than the base count
    to fill the last round of work items (20k x 20k: 19 splits on the MXFP4
    path instead of 9; 100k x 100k: 21 instead of 7): every row equals the
    batched matcher, which scans each pair's whole train range with no splits
    or merge, and a sample equals the oracle."""
    from paper_1609_03986_amd.binding import pair_table
    torch = torch_cuda
    g = np.random.default_rng(nq + nt)
    Q = synth.random_descriptors(g, nq, 0.3)
    T = synth.random_descriptors(g, nt, 0.3)
    T[7:17] = T[nt - 10:]                            # duplicate rows: ties across splits
    q, t = to_dev(torch, Q), to_dev(torch, T)
    lat.reserve(lat.knn_workspace_size(nq, nt, path))
    idx, dist, acc = lat.knn(q, t, path=path)
    both = torch.cat([q, t])
    b_idx, b_dist, b_acc = lat.knn_batch(both, both, pair_table([(0, nq, nq, nt, 0)]), nq, path=path)
    torch.cuda.synchronize()
    assert lat.check_errors(clear=True) == 0
    assert torch.equal(idx, b_idx) and torch.equal(dist, b_dist) and torch.equal(acc, b_acc)
    sel = np.arange(0, nq, 997)
    wi, wd, wa = oracle.knn(Q[sel], T)
    assert np.array_equal(idx.cpu().numpy()[sel], wi)
    assert np.array_equal(dist.cpu().numpy()[sel], wd)
    assert np.array_equal(acc.cpu().numpy()[sel], wa)
