"""GPU checks of hamming_knn_noalloc, the allocation-free matcher entry point:
its split partials live in the library's static device scratch, so it needs
no reservation.  Through the C ABI it gives exactly what hamming_knn gives
(and the oracle), on two calls in a row with the second smaller, refuses a
call whose partials exceed the scratch before enqueuing anything, and replays
correctly from a captured HIP graph."""
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


def outputs(torch, nq, fill=-7):
    idx = torch.full((nq, 2), fill, dtype=torch.int32, device="cuda")
    dist = torch.full((nq, 2), fill, dtype=torch.int32, device="cuda")
    acc = torch.full((nq,), 9, dtype=torch.uint8, device="cuda")
    return idx, dist, acc


def raw_call(torch, name, lat, q, t, idx, dist, acc, path, stream=None):
    """hamming_knn or hamming_knn_noalloc straight through ctypes."""
    from paper_1609_03986_amd import binding
    fn = getattr(binding.load_library(), name)
    s = stream if stream is not None else torch.cuda.current_stream()
    return fn(lat.h, ctypes.c_void_p(q.data_ptr()), q.shape[0], ctypes.c_void_p(t.data_ptr()),
              t.shape[0], 2, 0.8, ctypes.c_void_p(idx.data_ptr()),
              ctypes.c_void_p(dist.data_ptr()), ctypes.c_void_p(acc.data_ptr()),
              binding.PATHS[path], ctypes.c_void_p(s.cuda_stream))


def reference(torch, ref, q, t, path):
    """hamming_knn on a handle whose workspace is reserved for the call."""
    from paper_1609_03986_amd import binding
    ref.reserve(ref.knn_workspace_size(q.shape[0], t.shape[0], path))
    idx, dist, acc = outputs(torch, q.shape[0], fill=-5)
    assert raw_call(torch, "hamming_knn", ref, q, t, idx, dist, acc, path) == binding.LATCH_OK
    return idx, dist, acc


@pytest.mark.parametrize("path", ["fp4", "mfma", "popcount"])
def test_noalloc_equals_hamming_knn_on_two_calls(torch_cuda, triplets, path):
    torch = torch_cuda
    from paper_1609_03986_amd import binding
    from paper_1609_03986_amd.binding import Latch
    g = np.random.default_rng(77)
    lat, ref = Latch(triplets), Latch(triplets)
    try:
        assert lat.reserve(0) == 0                      # this handle never holds a workspace
        for call, (nq, nt) in enumerate([(3000, 40000), (700, 20000)]):
            Q = synth.random_descriptors(g, nq)
            T = synth.random_descriptors(g, nt, p_one=0.5 if call == 0 else 0.05)
            Q[:40] = T[nt - 40:]                         # exact matches at the end of the train set
            T[5:25] = T[1000:1020]                       # duplicate rows: ties to the lower index
            need = lat.knn_workspace_size(nq, nt, path)
            assert 0 < need <= binding.NOALLOC_SCRATCH_BYTES   # several splits, inside the scratch
            q, t = to_dev(torch, Q), to_dev(torch, T)
            idx, dist, acc = outputs(torch, nq)
            assert raw_call(torch, "hamming_knn_noalloc", lat, q, t, idx, dist, acc, path) == \
                binding.LATCH_OK
            ri, rd, ra = reference(torch, ref, q, t, path)
            torch.cuda.synchronize()
            assert torch.equal(idx, ri), (call, path)
            assert torch.equal(dist, rd), (call, path)
            assert torch.equal(acc, ra), (call, path)
            if call == 1:
                wi, wd, wa = oracle.knn(Q, T, k=2, ratio=0.8)
                assert np.array_equal(idx.cpu().numpy(), wi)
                assert np.array_equal(dist.cpu().numpy(), wd)
                assert np.array_equal(acc.cpu().numpy(), wa)
        assert lat.reserve(0) == 0                      # still no workspace
        assert lat.check_errors() == 0
    finally:
        torch.cuda.synchronize()
        lat.close()
        ref.close()


def test_noalloc_refuses_more_than_its_scratch(torch_cuda, triplets):
    torch = torch_cuda
    from paper_1609_03986_amd import binding
    from paper_1609_03986_amd.binding import Latch
    g = np.random.default_rng(5)
    nq, nt = 300000, 100000
    lat = Latch(triplets)
    try:
        # The MXFP4 path splits 100,000 train rows at least 7 ways: 16 bytes per
        # (query, split) is more than the scratch holds.
        assert lat.knn_workspace_size(nq, nt, "fp4") > binding.NOALLOC_SCRATCH_BYTES
        q = to_dev(torch, g.integers(0, 2**32, size=(nq, 16), dtype=np.uint32))
        t = to_dev(torch, g.integers(0, 2**32, size=(nt, 16), dtype=np.uint32))
        idx, dist, acc = outputs(torch, nq)
        rc = raw_call(torch, "hamming_knn_noalloc", lat, q, t, idx, dist, acc, "fp4")
        assert rc == binding.LATCH_ERANGE
        assert b"scratch" in binding.load_library().latch_last_error(lat.h)
        torch.cuda.synchronize()
        assert (idx == -7).all() and (dist == -7).all() and (acc == 9).all()   # nothing ran
        # A smaller call right after works.
        q2, t2 = q[:2000], t[:30000]
        idx2, dist2, acc2 = outputs(torch, 2000)
        assert raw_call(torch, "hamming_knn_noalloc", lat, q2, t2, idx2, dist2, acc2, "fp4") == \
            binding.LATCH_OK
        torch.cuda.synchronize()
        wi, wd, wa = oracle.knn(q2.cpu().numpy().view(np.uint32), t2.cpu().numpy().view(np.uint32),
                                k=2, ratio=0.8)
        assert np.array_equal(idx2.cpu().numpy(), wi)
        assert np.array_equal(dist2.cpu().numpy(), wd)
        assert np.array_equal(acc2.cpu().numpy(), wa)
    finally:
        torch.cuda.synchronize()
        lat.close()


def test_noalloc_keeps_extra_splits_within_its_scratch(torch_cuda, triplets):
    """16,000 queries against 1,000,000 rows: the split planner of hamming_knn
    adds splits beyond its base count to fill the last round of workgroups,
    and their partials would exceed the scratch; the allocation-free call adds
    only as many as fit.  It runs, and both give the same results (which never
    depend on the split count), equal to the oracle on a sample."""
    torch = torch_cuda
    from paper_1609_03986_amd import binding
    from paper_1609_03986_amd.binding import Latch
    g = np.random.default_rng(41)
    nq, nt = 16_000, 1_000_000
    lat, ref = Latch(triplets), Latch(triplets)
    try:
        assert ref.knn_workspace_size(nq, nt, "fp4") > binding.NOALLOC_SCRATCH_BYTES
        Q = synth.random_descriptors(g, nq)
        T = synth.random_descriptors(g, nt)
        Q[:20] = T[nt - 20:]                             # exact matches in the last split
        q, t = to_dev(torch, Q), to_dev(torch, T)
        idx, dist, acc = outputs(torch, nq)
        assert raw_call(torch, "hamming_knn_noalloc", lat, q, t, idx, dist, acc, "fp4") == \
            binding.LATCH_OK
        ri, rd, ra = reference(torch, ref, q, t, "fp4")
        torch.cuda.synchronize()
        assert torch.equal(idx, ri) and torch.equal(dist, rd) and torch.equal(acc, ra)
        sel = np.concatenate([np.arange(5), np.arange(20, nq, 1601)])
        wi, wd, wa = oracle.knn(Q[sel], T)
        assert np.array_equal(idx.cpu().numpy()[sel], wi)
        assert np.array_equal(dist.cpu().numpy()[sel], wd)
        assert np.array_equal(acc.cpu().numpy()[sel], wa)
        assert lat.check_errors() == 0
    finally:
        torch.cuda.synchronize()
        lat.close()
        ref.close()


def test_noalloc_captured_in_a_graph(torch_cuda, triplets):
    """Captured with no reservation at all; replays with new query contents
    and eager work between them, each equal to eager hamming_knn."""
    torch = torch_cuda
    from paper_1609_03986_amd import binding
    from paper_1609_03986_amd.binding import Latch
    g = np.random.default_rng(31)
    nq, nt = 1500, 36000
    T = synth.random_descriptors(g, nt)
    lat, ref = Latch(triplets), Latch(triplets)
    try:
        q = torch.zeros((nq, 16), dtype=torch.int32, device="cuda")
        t = to_dev(torch, T)
        idx, dist, acc = outputs(torch, nq)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            assert raw_call(torch, "hamming_knn_noalloc", lat, q, t, idx, dist, acc, "fp4",
                            stream=side) == binding.LATCH_OK
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            rc = raw_call(torch, "hamming_knn_noalloc", lat, q, t, idx, dist, acc, "fp4",
                          stream=torch.cuda.current_stream())
        assert rc == binding.LATCH_OK
        for rep in range(3):
            Q = synth.random_descriptors(g, nq, p_one=0.5 if rep != 1 else 0.05)
            Q[:30] = T[200 * rep:200 * rep + 30]
            q.copy_(to_dev(torch, Q))
            idx.fill_(-3)
            graph.replay()
            ri, rd, ra = reference(torch, ref, q, t, "fp4")
            torch.cuda.synchronize()
            assert torch.equal(idx, ri), rep
            assert torch.equal(dist, rd), rep
            assert torch.equal(acc, ra), rep
        del graph
    finally:
        torch.cuda.synchronize()
        lat.close()
        ref.close()
