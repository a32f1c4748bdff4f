"""GPU parity at the full sizes of the batched workloads (the SfM batch: 64
crops of 3000x2000 with 20,000 keypoints each and 63 consecutive 20k x 20k
pairs; the uneven batch: 256 images of the size mix, log-normal keypoint
counts), in one batched extraction and one batched matching launch (eager
calls, or one captured plan replayed twice): every descriptor against the
oracle's extraction (1.28 M and 1.91 M descriptors; the oracle's result is
computed once per workload) and 10,000 sampled queries against the oracle's
brute force over their pair's whole train range."""
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


_ORACLE_DESC = {}


def oracle_descriptors(name, imgs, kps, triplets):
    """The oracle's descriptors of every keypoint of a workload, in batch order."""
    if name not in _ORACLE_DESC:
        parts = []
        for im, k in zip(imgs, kps):
            d, f = oracle.extract(im, np.asarray(k, np.float32), triplets)
            assert f == 0
            parts.append(d)
        _ORACLE_DESC[name] = np.concatenate(parts)
    return _ORACLE_DESC[name]


def run_full(torch, triplets, imgs, kps, seed, name, plan=False):
    """Batched extraction and matching of the whole workload (eager calls, or
    one captured plan replayed twice), then every descriptor and sampled
    queries against the oracle."""
    from paper_1609_03986_amd.binding import Latch, image_table, pair_table
    lat = Latch(triplets)
    try:
        counts = [len(k) for k in kps]
        first = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
        total = int(sum(counts))
        dimgs = [torch.from_numpy(im).cuda() for im in imgs]
        kp_all = np.concatenate(kps).astype(np.float32)
        ids = np.repeat(np.arange(len(imgs), dtype=np.int32), counts)
        pairs = np.array([(first[i], counts[i], first[i + 1], counts[i + 1], first[i])
                          for i in range(len(imgs) - 1)], np.int64)
        table = image_table(dimgs)
        ids_d = torch.from_numpy(ids).cuda()
        kps_d = torch.from_numpy(kp_all).cuda()
        if plan:
            desc = torch.full((total, 16), -7, dtype=torch.int32, device="cuda")
            idx = torch.full((total, 2), -7, dtype=torch.int32, device="cuda")
            dist = torch.full((total, 2), -7, dtype=torch.int32, device="cuda")
            acc = torch.full((total,), 9, dtype=torch.uint8, device="cuda")
            p = lat.plan(table, len(imgs), ids_d, kps_d, desc, pair_table(pairs), idx, dist, acc)
            p.run()
            torch.cuda.synchronize()
            first_run = (desc.clone(), idx.clone(), dist.clone(), acc.clone())
            desc.fill_(-7)
            idx.fill_(-7)
            p.run()                                           # a replay gives the same outputs
            torch.cuda.synchronize()
            assert all(torch.equal(a, b) for a, b in zip(first_run, (desc, idx, dist, acc)))
            p.close()
        else:
            desc = lat.extract_batch(table, len(imgs), ids_d, kps_d)
            idx, dist, acc = lat.knn_batch(desc, desc, pair_table(pairs), total)
        torch.cuda.synchronize()
        assert lat.check_errors(clear=True) == 0
        D = desc.cpu().numpy().view(np.uint32)
        idx, dist, acc = idx.cpu().numpy(), dist.cpu().numpy(), acc.cpu().numpy()
    finally:
        lat.close()
    g = np.random.default_rng(seed)
    want = oracle_descriptors(name, imgs, kps, triplets)
    bad = np.nonzero((D != want).any(axis=1))[0]
    assert len(bad) == 0, (len(bad), bad[:10], ids[bad[:10]])
    # 10,000 queries of the pairs (queries of the last image have no pair).
    q_sel = np.sort(g.choice(first[-1], 10_000, replace=False))
    for i in np.unique(ids[q_sel]):
        qs = q_sel[ids[q_sel] == i]
        tf, nt = first[i + 1], counts[i + 1]
        wi, wd, wa = oracle.knn(D[qs], D[tf:tf + nt])
        assert np.array_equal(idx[qs], wi), int(i)
        assert np.array_equal(dist[qs], wd), int(i)
        assert np.array_equal(acc[qs], wa), int(i)


def test_sfm_batch_full_size(torch_cuda, triplets):
    imgs, kps = synth.sfm_workload()
    assert len(imgs) == 64 and imgs[0].shape == (2000, 3000) and len(kps[0]) == 20000
    run_full(torch_cuda, triplets, imgs, kps, 1, "sfm")


def test_uneven_batch_full_size(torch_cuda, triplets):
    imgs, kps = synth.uneven_workload()
    assert len(imgs) == 256
    run_full(torch_cuda, triplets, imgs, kps, 2, "uneven")


def test_sfm_batch_full_size_captured_plan(torch_cuda, triplets):
    imgs, kps = synth.sfm_workload()
    run_full(torch_cuda, triplets, imgs, kps, 3, "sfm", plan=True)


def test_uneven_batch_full_size_captured_plan(torch_cuda, triplets):
    imgs, kps = synth.uneven_workload()
    run_full(torch_cuda, triplets, imgs, kps, 4, "uneven", plan=True)
