"""The segmented sort behind the neighbour and core orders, through its
diagnostic entry point: every segment sorted by key descending, ties by id
ascending, for segment lengths across every size class of the sort (single
elements, lane groups of 8..64, blocks of 128..4096, several tiles merged in 1..5
passes, with segments of different pass counts in one call), with many tied
keys. Expected order: numpy's lexsort."""

from __future__ import annotations

import numpy as np
import pytest

import paper_2012_11188_amd as scan
from gpu_util import bits

pytestmark = pytest.mark.gpu

# Both sides of every class boundary (1, 8, 16, 32, 64, 128, ..., 4096).
EDGE_LENGTHS = [0, 1, 2, 3, 7, 8, 9, 15, 16, 17, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129, 255, 256, 257,
                511, 512, 513, 1000, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193,
                12289, 16384, 16385, 18859, 18859, 18859, 33000, 70001, 131072]


def make(lengths, seed, distinct_keys):
    rng = np.random.default_rng(seed)
    seg_off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    total = int(seg_off[-1])
    grid = rng.random(distinct_keys) + 1e-3  # few distinct keys: many ties
    keys = grid[rng.integers(0, distinct_keys, total)]
    ids = np.empty(total, np.int32)
    for i, ln in enumerate(lengths):
        ids[seg_off[i]:seg_off[i + 1]] = rng.choice(max(4 * ln, 1), ln, replace=False)
    return seg_off, keys, ids


def expected(seg_off, keys, ids):
    ko, io = np.empty_like(keys), np.empty_like(ids)
    for i in range(len(seg_off) - 1):
        b, e = seg_off[i], seg_off[i + 1]
        p = np.lexsort((ids[b:e], -keys[b:e]))
        ko[b:e], io[b:e] = keys[b:e][p], ids[b:e][p]
    return ko, io


@pytest.mark.parametrize("distinct", [3, 50, 10**6])
def test_segsort_edge_lengths(distinct):
    seg_off, keys, ids = make(EDGE_LENGTHS, seed=distinct, distinct_keys=distinct)
    ko, io = scan.scan_segmented_sort(seg_off, keys, ids)
    wk, wi = expected(seg_off, keys, ids)
    bad = np.flatnonzero(io != wi)
    if len(bad):
        seg = np.searchsorted(seg_off, bad[0], side="right") - 1
        pytest.fail(f"{len(bad)} ids differ; first at {bad[0]} in segment {seg} of length "
                    f"{seg_off[seg + 1] - seg_off[seg]}")
    assert np.array_equal(bits(ko), bits(wk))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_segsort_random_mix(seed):
    rng = np.random.default_rng(seed)
    small = rng.integers(0, 80, 3000)
    mid = rng.integers(65, 4097, 60)
    big = rng.integers(4097, 40000, 12)
    lengths = rng.permutation(np.concatenate([small, mid, big]))
    seg_off, keys, ids = make(lengths, seed=seed, distinct_keys=int(rng.integers(2, 1000)))
    ko, io = scan.scan_segmented_sort(seg_off, keys, ids)
    wk, wi = expected(seg_off, keys, ids)
    assert np.array_equal(io, wi) and np.array_equal(bits(ko), bits(wk))


def test_segsort_repeatable():
    seg_off, keys, ids = make([18859] * 40 + [5000] * 20 + [70] * 500, seed=9, distinct_keys=40)
    first = scan.scan_segmented_sort(seg_off, keys, ids)
    for _ in range(3):
        again = scan.scan_segmented_sort(seg_off, keys, ids)
        assert np.array_equal(again[1], first[1])
    assert np.array_equal(first[1], expected(seg_off, keys, ids)[1])


def test_segsort_errors():
    with pytest.raises(scan.ScanError):
        scan.scan_segmented_sort(np.array([0, 2, 1]), np.ones(2), np.arange(2))
    with pytest.raises(scan.ScanError):
        scan.scan_segmented_sort(np.array([0, 2]), np.array([1.0, np.nan]), np.arange(2))
    with pytest.raises(scan.ScanError):
        scan.scan_segmented_sort(np.array([0, 2]), np.array([1.0, -0.0]), np.arange(2))
    with pytest.raises(scan.ScanError):
        scan.scan_segmented_sort(np.array([0, 1]), np.array([1.0]), np.array([2**31 - 1]))


def test_segsort_negative_keys():
    # approximate similarities (cos(pi h / k)) can be negative: signed keys
    # in every segment class, with ties
    lengths = [1, 7, 33, 64, 65, 300, 1024, 1025, 4097, 9000]
    seg_off, keys, ids = make(lengths, 9, 40)
    keys = keys - 0.6  # about 60% negative
    assert (keys < 0).any() and (keys > 0).any()
    ko, io = scan.scan_segmented_sort(seg_off, keys, ids)
    eko, eio = expected(seg_off, keys, ids)
    assert np.array_equal(ko, eko) and np.array_equal(io, eio)


def test_segsort_partitioned_long_segments():
    # segments long enough for hundreds to thousands of buckets (the bucket
    # count is capped at 4096, so the 9M segment has buckets of ~2.2k), next
    # to short ones, with few distinct keys (ties broken by id across buckets)
    lengths = [3, 300_000, 64, 1_000_003, 5000, 1, 9_000_000, 4097]
    for distinct in (7, 10**6):
        seg_off, keys, ids = make(lengths, seed=distinct + 1, distinct_keys=distinct)
        ko, io = scan.scan_segmented_sort(seg_off, keys, ids)
        wk, wi = expected(seg_off, keys, ids)
        assert np.array_equal(io, wi), distinct
        assert np.array_equal(bits(ko), bits(wk)), distinct


def test_segsort_partition_with_skewed_samples():
    # every sampled position of a 100,000-element segment holds the smallest
    # key, so every splitter does too: all other elements fall into the first
    # bucket, far over 4096, which must then be sorted by the merge path
    n, S = 100_000, 16 * ((100_000 + 2047) // 2048)
    rng = np.random.default_rng(4)
    keys = 0.6 + 0.4 * rng.random(n)
    pos = ((2 * np.arange(S) + 1) * n) // (2 * S)
    keys[pos] = 0.5
    ids = rng.choice(4 * n, n, replace=False).astype(np.int32)
    seg_off = np.array([0, 7, 7 + n, 7 + n + 5], np.int64)
    keys = np.concatenate([rng.random(7) + 0.1, keys, rng.random(5) + 0.1])
    ids = np.concatenate([np.arange(7, dtype=np.int32), ids, np.arange(5, dtype=np.int32)])
    ko, io = scan.scan_segmented_sort(seg_off, keys, ids)
    wk, wi = expected(seg_off, keys, ids)
    assert np.array_equal(io, wi) and np.array_equal(bits(ko), bits(wk))


def test_segsort_all_keys_equal():
    # one key everywhere: the order is the id order alone, in every class
    lengths = [1, 40, 900, 4096, 4097, 70_000, 250_000]
    seg_off, keys, ids = make(lengths, seed=12, distinct_keys=1)
    ko, io = scan.scan_segmented_sort(seg_off, keys, ids)
    wk, wi = expected(seg_off, keys, ids)
    assert np.array_equal(io, wi) and np.array_equal(bits(ko), bits(wk))
