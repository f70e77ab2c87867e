"""Pins of the oracle's hash table: section "Hash Table and Hashing Function" and
section "Hash Table Operations" of the paper."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hash_index.txt")


def _golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(tuple(int(t) for t in line.split()))
    return rows


@pytest.mark.parametrize("row", _golden_rows())
def test_hash_index_hand_values(orc, row):
    x, y, z, mask, expected = row
    assert orc.hash_index(x, y, z, mask) == expected


def test_hash_index_mask_nesting(orc):
    # masking with a smaller power of two keeps the low bits of a larger mask's result
    rng = np.random.default_rng(5)
    for x, y, z in rng.integers(-3000, 3000, size=(200, 3)):
        big = orc.hash_index(int(x), int(y), int(z), 2 ** 22 - 1)
        assert orc.hash_index(int(x), int(y), int(z), 2 ** 14 - 1) == big & (2 ** 14 - 1)


def _walk(pos, off, ptr, n_buckets, key, hash_fn):
    """Retrieval written from the section's prose: check the bucket, then follow
    the offsets of the excess list; returns (entry, entries visited)."""
    base = hash_fn(*key) * 2
    seen = []
    for i in range(2):
        seen.append(base + i)
        if tuple(pos[base + i]) == key and ptr[base + i] >= 0:
            return base + i, seen
    o = off[base + 1] - 1
    while o >= 0:
        idx = 2 * n_buckets + o
        assert idx not in seen, "cycle in an excess chain"
        seen.append(idx)
        if tuple(pos[idx]) == key and ptr[idx] >= 0:
            return idx, seen
        o = off[idx] - 1
    return -1, seen


def test_insert_retrieve_with_excess_chains(orc):
    # 4 buckets of 2 entries + 40 excess entries: most keys land in chains
    nb, nx = 4, 40
    sc = orc.Scene(0.01, 0.04, 100, nb, nx)
    rng = np.random.default_rng(11)
    keys = {tuple(int(v) for v in k) for k in rng.integers(-50, 50, size=(40, 3))}
    keys = sorted(keys)[:46]
    inserted = {}
    for k in keys:
        e = sc.insert(*k)
        if e >= 0:
            inserted[k] = e
    st = sc.stats()
    # capacity: 2 per bucket plus the excess list
    per_bucket = {}
    for k in keys:
        h = orc.hash_index(*k, nb - 1)
        per_bucket[h] = per_bucket.get(h, 0) + 1
    demand = sum(max(0, n - 2) for n in per_bucket.values())
    assert st["excess_demand"] == min(demand, nx)
    assert st["n_allocated"] == sum(min(n, 2) for n in per_bucket.values()) + min(demand, nx)
    pos, off, ptr = sc.entries()
    for k, e in inserted.items():
        assert sc.find(*k) == e
        got, _ = _walk(pos, off, ptr, nb, k, lambda x, y, z: orc.hash_index(x, y, z, nb - 1))
        assert got == e
    # a key that was never inserted is not found
    assert sc.find(999, 999, 999) == -1
    # re-insertion returns the existing entry and allocates nothing new
    n0 = sc.stats()["n_allocated"]
    for k, e in inserted.items():
        assert sc.insert(*k) == e
    assert sc.stats()["n_allocated"] == n0


def test_excess_exhaustion_drops(orc):
    sc = orc.Scene(0.01, 0.04, 100, 1, 3)   # one bucket of 2, 3 excess entries
    got = [sc.insert(i, 0, 0) for i in range(8)]
    assert sum(g >= 0 for g in got) == 5
    assert got[5:] == [-1, -1, -1]
    assert sc.stats()["n_allocated"] == 5
