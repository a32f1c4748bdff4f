"""Autotuner: CPU tests of its selection logic and size buckets; a GPU test
that a measured tuning installs, round-trips, rejects bad entries, and never
changes results."""
import numpy as np
import pytest

import oracle
from paper_1609_03986_amd import autotune, synth
from paper_1609_03986_amd.binding import size_bucket


def test_size_bucket_is_half_log2():
    for n in [0, 1, 2, 3, 4, 5, 15, 16, 17, 255, 256, 1000, 4095, 4096, 16383, 16384, 10 ** 7]:
        want = 0 if n < 4 else min(7, int(np.floor(np.log2(n) / 2)))
        assert size_bucket(n) == want, n
    for b in range(8):
        assert size_bucket(autotune.bucket_shape(b)) == b


def test_choose_fastest_with_stable_ties():
    assert autotune.choose({1: 2.0, 2: 1.0}) == 2
    assert autotune.choose({1: 1.0, 2: 1.0}) == 1
    assert autotune.choose({3: 5.0, 1: 4.0, 2: 4.0}) == 1


def test_fill_table_nearest_measured_bucket():
    t = autotune.fill_table({(2, 2): 2, (6, 6): 1})
    assert t[0][0] == 2 and t[2][3] == 2 and t[7][7] == 1 and t[5][6] == 1
    assert autotune.fill_table({}) == [[3] * 8 for _ in range(8)]     # the library default, MXFP4


@pytest.mark.gpu
def test_tuning_roundtrip_and_results_unchanged(triplets):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_03986_amd.binding import Latch, LatchError, Tuning
    lat = Latch(triplets)
    try:
        t = autotune.tune(lat, buckets=[(2, 6), (6, 6)], reps=2)
        got = lat.get_tuning().to_dict()
        assert got == t
        bad = dict(t)
        bad["mfma_groups_per_cu"] = 0
        with pytest.raises(LatchError):
            lat.set_tuning(Tuning.from_dict(bad))
        bad = dict(t)
        bad["path"] = [row[:] for row in t["path"]]
        bad["path"][3][3] = 0
        with pytest.raises(LatchError):
            lat.set_tuning(Tuning.from_dict(bad))
        assert lat.get_tuning().to_dict() == t          # unchanged by rejected sets
        g = np.random.default_rng(3)
        for nq, nt in [(20, 5000), (3000, 3000), (700, 70)]:
            Q = synth.random_descriptors(g, nq)
            T = synth.random_descriptors(g, nt)
            for code in (1, 2, 3):                         # force each path through the table
                forced = dict(t)
                forced["path"] = [[code] * 8 for _ in range(8)]
                lat.set_tuning(Tuning.from_dict(forced))
                i, d, a = lat.knn(torch.from_numpy(Q.view(np.int32)).cuda(),
                                  torch.from_numpy(T.view(np.int32)).cuda(), path="auto")
                torch.cuda.synchronize()
                wi, wd, wa = oracle.knn(Q, T)
                assert np.array_equal(i.cpu().numpy(), wi) and np.array_equal(d.cpu().numpy(), wd)
                assert np.array_equal(a.cpu().numpy(), wa)
    finally:
        lat.close()
