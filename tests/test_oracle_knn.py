"""Pins for the oracle's Hamming distance and brute-force 2-NN matcher.

The paper matches binary descriptors exhaustively under Hamming distance
(Sec. 4, "Descriptor matching on the GPU") without stating k, the ratio test
or ties; the library fixes k = 2, ties to the lowest train index and
accept = d1 < ratio * d2 evaluated exactly.  Pinned against numpy bit
unpacking, a full lexicographic sort, metric axioms and hand-built distances.
"""
import numpy as np
import pytest

import oracle
from paper_1609_03986_amd import synth


def bits(d):
    return np.unpackbits(np.ascontiguousarray(d, np.uint32).view(np.uint8), axis=-1,
                         bitorder="little").astype(np.int64)


def test_hamming_axioms():
    g = np.random.default_rng(0)
    D = synth.random_descriptors(g, 40)
    for i in range(40):
        assert oracle.hamming(D[i], D[i]) == 0
        assert oracle.hamming(D[i], ~D[i]) == 512
        for j in range(0, 40, 7):
            dij = oracle.hamming(D[i], D[j])
            assert dij == oracle.hamming(D[j], D[i])
            for k in range(0, 40, 11):
                assert dij <= oracle.hamming(D[i], D[k]) + oracle.hamming(D[k], D[j])


def test_hamming_equals_unpacked_bits_and_dot_identity():
    g = np.random.default_rng(1)
    A = synth.random_descriptors(g, 30, 0.3)
    B = synth.random_descriptors(g, 30, 0.7)
    A[0] = 0
    B[1] = 0xFFFFFFFF
    ba, bb = bits(A), bits(B)
    dot = ba @ bb.T                                  # int64 matmul over {0,1}
    ham = ba.sum(1)[:, None] + bb.sum(1)[None, :] - 2 * dot
    for i in range(30):
        for j in range(30):
            assert oracle.hamming(A[i], B[j]) == int(np.count_nonzero(ba[i] != bb[j]))
            assert oracle.hamming(A[i], B[j]) == int(ham[i, j])


def full_sort_knn(Q, T, k):
    bq, bt = bits(Q), bits(T)
    idx = np.full((len(Q), k), -1, np.int32)
    dist = np.full((len(Q), k), 513, np.int32)
    for q in range(len(Q)):
        d = (bq[q][None, :] != bt).sum(1)
        order = np.lexsort((np.arange(len(T)), d))   # by distance, then by index
        for r in range(min(k, len(T))):
            idx[q, r] = order[r]
            dist[q, r] = d[order[r]]
    return idx, dist


@pytest.mark.parametrize("seed", range(12))
def test_knn_against_full_sort(seed):
    g = np.random.default_rng(seed)
    nq, nt = int(g.integers(1, 17)), int(g.integers(0, 17))
    p = float(g.choice([0.5, 0.05, 0.01]))          # sparse bits -> many ties
    Q = synth.random_descriptors(g, nq, p)
    T = synth.random_descriptors(g, nt, p) if nt else np.zeros((0, 16), np.uint32)
    if nt > 3:
        T[2] = T[0]                                   # exact duplicates
    for k in (1, 2):
        idx, dist, acc = oracle.knn(Q, T, k=k, ratio=0.8)
        ri, rd = full_sort_knn(Q, T, k)
        assert np.array_equal(idx, ri)
        assert np.array_equal(dist, rd)


def test_self_match_and_duplicates_resolve_to_lowest_index():
    g = np.random.default_rng(5)
    T = synth.random_descriptors(g, 20)
    T[11] = T[4]
    idx, dist, _ = oracle.knn(T, T, k=2)
    assert np.all(dist[:, 0] == 0)
    want = np.arange(20)
    want[11] = 4
    assert np.array_equal(idx[:, 0], want)
    assert idx[4, 1] == 11 and dist[4, 1] == 0


def with_popcount(n_bits_list):
    out = np.zeros((len(n_bits_list), 16), np.uint32)
    for r, n in enumerate(n_bits_list):
        b = np.zeros(512, np.uint8)
        b[:n] = 1
        out[r] = np.packbits(b, bitorder="little").view(np.uint32)
    return out


@pytest.mark.parametrize("d1,d2,ratio,want", [
    (4, 5, 0.8, 1),        # float32(0.8) = 0.800000011920929 > 4/5
    (8, 10, 0.8, 1),
    (3, 4, 0.75, 0),       # 0.75 is exact: 3 < 3 is false
    (0, 0, 0.8, 0),
    (0, 1, 0.8, 1),
    (7, 9, 0.8, 1),
    (9, 11, 0.8, 0),       # 9 < 8.8 is false
    (400, 500, 0.8, 1),
    (401, 500, 0.8, 0),
    (5, 5, 1.0, 0),
])
def test_ratio_test_edges(d1, d2, ratio, want):
    Q = np.zeros((1, 16), np.uint32)
    T = with_popcount([d2, d1, 512])
    idx, dist, acc = oracle.knn(Q, T, k=2, ratio=ratio)
    if d1 < d2:
        assert list(idx[0]) == [1, 0]
    assert list(dist[0]) == [d1, d2]
    assert acc[0] == want


def test_fewer_than_two_train_rows():
    Q = synth.random_descriptors(np.random.default_rng(6), 3)
    idx, dist, acc = oracle.knn(Q, np.zeros((0, 16), np.uint32), k=2)
    assert np.all(idx == -1) and np.all(dist == 513) and not acc.any()
    idx, dist, acc = oracle.knn(Q, Q[:1], k=2)
    assert np.all(idx[:, 0] == 0) and np.all(idx[:, 1] == -1) and np.all(dist[:, 1] == 513)
    assert not acc.any()
    idx, dist, acc = oracle.knn(Q, Q[:1], k=1)
    assert idx.shape == (3, 1) and np.all(idx[:, 0] == 0)
