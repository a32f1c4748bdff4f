"""GPU serving test: requests served concurrently (several slots, overlapping
arrivals) get exactly the results they get alone, and those equal the oracle."""
import numpy as np
import pytest

import oracle
from paper_1609_03986_amd import serve, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_each_result_is_the_same_alone_and_in_the_mix(torch_cuda, triplets):
    torch = torch_cuda
    from paper_1609_03986_amd.binding import Latch
    g = np.random.default_rng(21)
    db_np = synth.random_descriptors(g, 20000)
    db = torch.from_numpy(db_np.view(np.int32)).cuda()
    sizes = [(240, 320), (480, 640), (720, 1280), (121, 97)]
    imgs = [synth.smoothed_noise(g, *hw) for hw in sizes]
    reqs = []
    for i in range(12):
        k = i % len(sizes)
        n = int(g.integers(100, 3000))
        reqs.append(serve.Request(i, imgs[k], synth.random_keypoints(g, n, *sizes[k]), 0.0005 * i))
    mixed_ex = serve.GpuExecutor(db, triplets, n_slots=4)
    mixed, rej, stats = serve.Scheduler(mixed_ex, 4, 1 << 32, len(db_np)).run(reqs)
    assert not rej and stats["served"] == 12
    assert stats["max_inflight"] > 1
    alone_ex = serve.GpuExecutor(db, triplets, n_slots=1)
    alone = {}
    for r in reqs:
        res, _, _ = serve.Scheduler(alone_ex, 1, 1 << 32, len(db_np)).run(
            [serve.Request(r.rid, r.image, r.kps, 0.0)])
        alone[r.rid] = res[0]
    for r in mixed:
        a = alone[r.rid]
        assert np.array_equal(r.idx, a.idx) and np.array_equal(r.dist, a.dist)
        assert np.array_equal(r.accept, a.accept)
    for rid in (0, 5, 11):
        q = reqs[rid]
        d, _ = oracle.extract(q.image, q.kps, triplets)
        wi, wd, wa = oracle.knn(d, db_np)
        m = [r for r in mixed if r.rid == rid][0]
        assert np.array_equal(m.idx, wi) and np.array_equal(m.dist, wd)
        assert np.array_equal(m.accept, wa)
    mixed_ex.close()
    alone_ex.close()


def test_full_size_database_sampled(torch_cuda, triplets):
    """The serving configuration: a resident 1,000,000-row database extracted
    on the GPU from 50 seeded 1920x1080 images, requests from the uneven mix.
    Every database row (the builder's images and keypoints regenerated from
    its seed) and 1,000 sampled queries (over three requests, each against the
    whole database) equal the oracle."""
    torch = torch_cuda
    from paper_1609_03986_amd.binding import Latch
    lat = Latch(triplets)
    try:
        db = serve.build_database(lat)
        assert db.shape == (1_000_000, 16)
        db_np = db.cpu().numpy().view(np.uint32)
        # The builder's images and keypoints, regenerated from its seed.
        g = np.random.default_rng(3)
        for i in range(50):
            img = synth.smoothed_noise(g, 1080, 1920)
            kps = synth.random_keypoints(g, 20000, 1080, 1920)
            want, f = oracle.extract(img, kps, triplets)
            assert f == 0 and np.array_equal(db_np[20000 * i:20000 * (i + 1)], want), i
        pool = serve.request_pool()
        reqs = serve.make_requests(3, 100.0, pool)
        ex = serve.GpuExecutor(db, triplets, n_slots=2)
        try:
            # Admission uses the library's own workspace figures: on the
            # default MXFP4 path a 1M-row database needs at least 62 splits
            # of 2^14 rows, 16 bytes per query and split, and every slot has
            # reserved the largest need of the mix up front.
            for n in (500, 5000, 25000, 50000):
                need = ex.workspace_need(n)
                assert need == lat.knn_workspace_size(n, 1_000_000, "auto")
                assert need >= 62 * 16 * n
                assert ex.workspace_bytes(n) == 0
            assert ex.reserved >= ex.workspace_need(50000)
            assert ex.retained_bytes() == 2 * ex.slots[0]["lat"].reserve(0) >= 2 * ex.reserved
            results, rej, stats = serve.Scheduler(ex, 2, 1 << 36, len(db_np)).run(reqs)
            assert ex.retained_bytes() == 2 * ex.slots[0]["lat"].reserve(0)   # nothing grew
        finally:
            ex.close()
        assert not rej and stats["served"] == 3
        rng = np.random.default_rng(4)
        n_total = sum(len(r.kps) for r in reqs)
        per = [max(1, round(1000 * len(r.kps) / n_total)) for r in reqs]
        for r, k in zip(reqs, per):
            m = [x for x in results if x.rid == r.rid][0]
            qs = np.sort(rng.choice(len(r.kps), min(k, len(r.kps)), replace=False))
            d, _ = oracle.extract(r.image, r.kps[qs], triplets)
            wi, wd, wa = oracle.knn(d, db_np)
            assert np.array_equal(m.idx[qs], wi) and np.array_equal(m.dist[qs], wd)
            assert np.array_equal(m.accept[qs], wa)
    finally:
        lat.close()
