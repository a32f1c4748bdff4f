"""GPU checks of the workspace contract of the C ABI: the work calls never
allocate or wait, a call whose workspace need exceeds what the handle holds
fails with LATCH_EWORKSPACE before it enqueues anything, latch_reserve sizes
the workspace to what the *_workspace_size calls report, and hamming_knn
captured in a HIP graph after a reservation replays to the oracle's results."""
import ctypes

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


def to_dev(torch, d):
    return torch.from_numpy(np.ascontiguousarray(d, np.uint32).view(np.int32)).cuda()


def raw_knn(torch, lat, q, t, idx, dist, acc, path):
    from paper_1609_03986_amd import binding
    lib = binding.load_library()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib.hamming_knn(lat.h, ctypes.c_void_p(q.data_ptr()), q.shape[0],
                           ctypes.c_void_p(t.data_ptr()), t.shape[0], 2, 0.8,
                           ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
                           ctypes.c_void_p(acc.data_ptr()), binding.PATHS[path], s)


@pytest.mark.parametrize("path", ["mfma", "fp4", "popcount"])
def test_too_small_workspace_is_an_error_then_reserve_fixes_it(torch_cuda, triplets, path):
    torch = torch_cuda
    from paper_1609_03986_amd import binding
    from paper_1609_03986_amd.binding import Latch
    g = np.random.default_rng(3)
    Q, T = synth.random_descriptors(g, 700), synth.random_descriptors(g, 30000)
    lat = Latch(triplets)
    try:
        need = lat.knn_workspace_size(len(Q), len(T), path)
        assert need > 0                                          # several train splits
        assert lat.reserve(0) == 0                               # a new handle holds none
        q, t = to_dev(torch, Q), to_dev(torch, T)
        idx = torch.full((len(Q), 2), -7, dtype=torch.int32, device="cuda")
        dist = torch.full((len(Q), 2), -7, dtype=torch.int32, device="cuda")
        acc = torch.full((len(Q),), 9, dtype=torch.uint8, device="cuda")
        assert raw_knn(torch, lat, q, t, idx, dist, acc, path) == binding.LATCH_EWORKSPACE
        assert b"latch_reserve" in binding.load_library().latch_last_error(lat.h)
        torch.cuda.synchronize()
        assert (idx == -7).all() and (dist == -7).all() and (acc == 9).all()   # nothing ran
        assert lat.reserve(need - 1) >= need - 1
        held = lat.reserve(need)
        assert held >= need and lat.reserve(0) == held
        assert raw_knn(torch, lat, q, t, idx, dist, acc, path) == binding.LATCH_OK
        torch.cuda.synchronize()
        wi, wd, wa = oracle.knn(Q, T, k=2, ratio=0.8)
        assert np.array_equal(idx.cpu().numpy(), wi)
        assert np.array_equal(dist.cpu().numpy(), wd)
        assert np.array_equal(acc.cpu().numpy(), wa)
        # A larger reservation replaces the buffer; a smaller one keeps it.
        assert lat.reserve(held + 4096) >= held + 4096
        assert lat.reserve(16) >= held + 4096
    finally:
        lat.close()


def test_workspace_sizes_follow_the_split_plan(torch_cuda, triplets):
    from paper_1609_03986_amd.binding import Latch
    lat = Latch(triplets)
    try:
        assert lat.knn_workspace_size(0, 5000) == 0
        assert lat.knn_workspace_size(100, 0) == 0
        # A 1M-row train set on the MXFP4 path: splits of at most 2^14 rows,
        # so at least 62 splits of 16 bytes per query.
        for nq in (500, 5000, 50000):
            b = lat.knn_workspace_size(nq, 1_000_000, "fp4")
            assert b >= 62 * nq * 16 and b % (nq * 16) < 256 + nq * 16
        assert lat.knn_batch_workspace_size(0, 100) == 0
        assert lat.knn_batch_workspace_size(63, 1_280_000) > 63 * 8
        assert lat.detect_workspace_size(1080, 1920) >= 8 * 1080 * 30 + 8 * 1080
    finally:
        lat.close()


def test_detect_needs_its_reservation(torch_cuda, triplets):
    torch = torch_cuda
    from paper_1609_03986_amd import binding
    from paper_1609_03986_amd.binding import Latch
    g = np.random.default_rng(8)
    img = synth.smoothed_noise(g, 120, 150)
    lat = Latch(triplets)
    try:
        lib = binding.load_library()
        dimg = torch.from_numpy(img).cuda()
        kps = torch.empty((4096, 4), dtype=torch.float32, device="cuda")
        n = torch.zeros((1,), dtype=torch.int64, device="cuda")
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        args = (lat.h, ctypes.c_void_p(dimg.data_ptr()), 120, 150, 150, 20,
                ctypes.c_void_p(kps.data_ptr()), 4096, ctypes.c_void_p(n.data_ptr()), None, 0, s)
        assert lib.latch_detect(*args) == binding.LATCH_EWORKSPACE
        lat.reserve(lat.detect_workspace_size(120, 150))
        assert lib.latch_detect(*args) == binding.LATCH_OK
        torch.cuda.synchronize()
        want, wn = oracle.detect(img, 20)
        assert int(n.item()) == wn and np.array_equal(kps[:wn].cpu().numpy(), want)
    finally:
        lat.close()


@pytest.mark.parametrize("path", ["fp4", "mfma"])
def test_captured_knn_replays_to_the_oracle(torch_cuda, triplets, path):
    """hamming_knn (split kernel + merge) captured into a graph after a
    reservation; replays with new query contents, eager work and
    synchronisations in between, each checked against the oracle."""
    torch = torch_cuda
    from paper_1609_03986_amd.binding import Latch
    g = np.random.default_rng(21)
    T = synth.random_descriptors(g, 20000)
    nq = 1000
    lat = Latch(triplets)
    other = Latch(triplets)
    try:
        lat.reserve(lat.knn_workspace_size(nq, len(T), path))
        q = torch.zeros((nq, 16), dtype=torch.int32, device="cuda")
        t = to_dev(torch, T)
        idx = torch.empty((nq, 2), dtype=torch.int32, device="cuda")
        dist = torch.empty((nq, 2), dtype=torch.int32, device="cuda")
        acc = torch.empty((nq,), dtype=torch.uint8, device="cuda")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            lat.knn(q, t, path=path, idx=idx, dist=dist, accept=acc)       # eager once
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            lat.knn(q, t, path=path, idx=idx, dist=dist, accept=acc)
        for rep in range(4):
            Q = synth.random_descriptors(g, nq, p_one=0.5 if rep % 2 == 0 else 0.05)
            if rep == 3:
                Q[:50] = T[100:150]                                  # exact matches
            q.copy_(to_dev(torch, Q))
            idx.fill_(-3)
            graph.replay()
            torch.cuda.synchronize()
            wi, wd, wa = oracle.knn(Q, T, k=2, ratio=0.8)
            assert np.array_equal(idx.cpu().numpy(), wi), rep
            assert np.array_equal(dist.cpu().numpy(), wd), rep
            assert np.array_equal(acc.cpu().numpy(), wa), rep
            # Eager work of the program between replays (on another handle:
            # the graph holds this handle's workspace address, which a
            # reservation that replaces the buffer would invalidate).
            other.knn(q, t[:5000], path="popcount")
            torch.cuda.synchronize()
        del graph
    finally:
        torch.cuda.synchronize()
        lat.close()
        other.close()
