"""Nearest-neighbour descriptor matching (sift3d_match) against the oracle's
brute force, exactly: index (lowest among equal distances), distance and
second-smallest distance, for binary BRIEF words and uint8 rank vectors,
with ragged sizes spanning several LDS tiles, duplicates (ties), an empty
and a one-row B, and the descriptors of a real extraction."""
import numpy as np
import pytest

import oracle as O
from gen import phantoms as P

pytestmark = pytest.mark.gpu


def _gpu_match(A, B, kind):
    import torch

    import paper_2112_10258_amd as S
    ta = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    tb = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    idx, d1, d2 = S.match(ta, tb, kind)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), d1.cpu().numpy(), d2.cpu().numpy()


def _same(A, B, kind, what):
    got = _gpu_match(A, B, kind)
    want = O.match_nn(A.view(np.uint64) if kind == 0 else A, B.view(np.uint64) if kind == 0 else B, kind)
    for g, w, name in zip(got, want, ("idx", "d1", "d2")):
        assert np.array_equal(g.astype(np.int64), w), (what, name)


@pytest.mark.parametrize("words", [1, 2, 3, 4])
def test_match_brief_words(words):
    import paper_2112_10258_amd as S
    rng = np.random.default_rng(100 + words)
    for n_a, n_b in ((1, 1), (300, 1500), (257, 0), (70, 2)):
        A = rng.integers(-2 ** 63, 2 ** 63 - 1, size=(n_a, words), dtype=np.int64)
        B = rng.integers(-2 ** 63, 2 ** 63 - 1, size=(n_b, words), dtype=np.int64)
        if n_b > 10:
            B[5] = B[3]                      # a tie: index 3 must win
            A[0] = B[3]
        _same(A, B, S.MATCH_BRIEF, (words, n_a, n_b))
    print(f"[match] brief {words} words: ok", flush=True)


@pytest.mark.parametrize("m", [64, 128, 192, 256])
def test_match_rank_vectors(m):
    import paper_2112_10258_amd as S
    rng = np.random.default_rng(200 + m)
    for n_a, n_b in ((1, 1), (333, 1100), (129, 0), (40, 2)):
        A = np.array([rng.permutation(m) for _ in range(n_a)], dtype=np.uint8).reshape(n_a, m)
        B = np.array([rng.permutation(m) for _ in range(n_b)], dtype=np.uint8).reshape(n_b, m)
        if n_b > 600:
            B[600] = B[7]                    # duplicate across LDS tiles: index 7 must win
            A[1] = B[7]
        _same(A, B, S.MATCH_RANKS, (m, n_a, n_b))
    print(f"[match] ranks {m}: ok", flush=True)


def test_match_extracted_descriptors():
    """SIFT-Rank, RRIEF and BRIEF of config 1 against a shuffled copy of
    themselves, and of config 1 against another volume."""
    import paper_2112_10258_amd as S
    from tests.helpers import gpu_extract
    g = gpu_extract(P.config1(), n_octaves=2, levels=False)
    h = gpu_extract(P.noise_blob_volume((60, 58, 62), 77, n_blobs=20, margin=6), min_dim=8, levels=False)
    rng = np.random.default_rng(5)
    perm = rng.permutation(g["count"])
    for f, kind in (("siftrank", S.MATCH_RANKS), ("rrief", S.MATCH_RANKS), ("brief", S.MATCH_BRIEF)):
        A = g[f] if kind == S.MATCH_RANKS else g[f].view(np.int64)
        Bh = h[f] if kind == S.MATCH_RANKS else h[f].view(np.int64)
        _same(A, A[perm], kind, f)
        _same(A, Bh, kind, f + " vs other volume")
    print(f"[match] extracted descriptors: {g['count']} vs {h['count']} keypoints ok", flush=True)


@pytest.mark.parametrize("m", [64, 256])
def test_match_rank_rows_with_many_ties_and_extreme_bytes(m):
    """Rows drawn from a small pool (many exact ties inside one tile, across
    the two halves of a lane pair and across wavefronts and tiles) and bytes
    at both ends of 0..255, with more A rows than one workgroup's block."""
    import paper_2112_10258_amd as S
    rng = np.random.default_rng(300 + m)
    pool = rng.integers(0, 256, size=(40, m), dtype=np.uint8)
    pool[0] = 0
    pool[1] = 255
    n_a, n_b = 1000, 2600
    A = pool[rng.integers(0, 40, n_a)]
    B = pool[rng.integers(0, 40, n_b)]
    _same(A, B, S.MATCH_RANKS, ("pool", m))
    print(f"[match] ranks {m}: pool rows with ties ok", flush=True)


def test_match_at_benchmark_size_on_sampled_rows():
    """16384 x 16384, the size the benchmark times (64-element rank vectors
    as random permutations, 4-word BRIEF rows): every A row is matched on
    the GPU; sampled rows (the first, the last, and random ones) equal the
    oracle's brute force exactly."""
    import paper_2112_10258_amd as S
    n = 16384
    rng = np.random.default_rng(2112)
    cases = (
        (S.MATCH_RANKS, np.argsort(rng.random((n, 64)), axis=1).astype(np.uint8),
         np.argsort(rng.random((n, 64)), axis=1).astype(np.uint8), 300),
        (S.MATCH_BRIEF, rng.integers(-2 ** 63, 2 ** 63 - 1, size=(n, 4), dtype=np.int64),
         rng.integers(-2 ** 63, 2 ** 63 - 1, size=(n, 4), dtype=np.int64), 60),
    )
    for kind, A, B, n_pick in cases:
        got = _gpu_match(A, B, kind)
        pick = np.unique(np.concatenate([[0, n - 1], rng.choice(n, n_pick, replace=False)]))
        sub = A[pick]
        want = O.match_nn(sub.view(np.uint64) if kind == S.MATCH_BRIEF else sub,
                          B.view(np.uint64) if kind == S.MATCH_BRIEF else B, kind)
        for g, w, name in zip(got, want, ("idx", "d1", "d2")):
            assert np.array_equal(g[pick].astype(np.int64), w), (kind, name)
        assert got[0].min() >= 0 and got[0].max() < n
        assert np.all(got[1] <= got[2])
