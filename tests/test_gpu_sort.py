"""Parity of the radix sort that orders every index curve (Section II.C: a
curve's entries by curve position), called directly through the C ABI on
seeded multi-word keys and checked against numpy's stable lexicographic
sort: keys ascending, equal keys in input order. The cases cover every path
of the sort: one key word, several varying words (passes on ranks with
gathers between words), several words of which only one varies, duplicate
keys, digit positions constant over the arrays (skipped), ragged lengths
around the 4096-item tile, several arrays in one call, and four words."""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _reference(keys, ids):
    """numpy's stable sort of each array by its key words (word 0 first)."""
    arrays, words, n = keys.shape
    ko, io = np.empty_like(keys), np.empty_like(ids)
    for a in range(arrays):
        order = np.lexsort(tuple(keys[a, w] for w in range(words - 1, -1, -1)))
        ko[a] = keys[a][:, order]
        io[a] = ids[a][order]
    return ko, io


def _run(keys, ids):
    nat = need_gpu()
    keys, ids = np.ascontiguousarray(keys), np.ascontiguousarray(ids)
    kd = torch.from_numpy(keys.view(np.int64)).cuda()
    idd = torch.from_numpy(ids.view(np.int32)).cuda()
    nat.sort_pairs(kd, idd)
    torch.cuda.synchronize()
    ko, io = _reference(keys, ids)
    assert np.array_equal(kd.cpu().numpy().view(np.uint64), ko)
    assert np.array_equal(idd.cpu().numpy().view(np.uint32), io)


def _keys(rng, arrays, words, n, top_bits=64):
    k = rng.integers(0, 2**63, size=(arrays, words, n), dtype=np.uint64) * np.uint64(2) \
        + rng.integers(0, 2, size=(arrays, words, n), dtype=np.uint64)
    if top_bits < 64:
        k[:, 0, :] &= np.uint64((1 << top_bits) - 1)
    return k


def _ids(arrays, n, ascending=True, rng=None):
    ids = np.tile(np.arange(n, dtype=np.uint32) * 3 + 5, (arrays, 1))
    if not ascending:
        for a in range(arrays):
            rng.shuffle(ids[a])
    return ids


@pytest.mark.parametrize("words,n,arrays,top", [
    (1, 4097, 2, 64), (2, 12345, 3, 16), (3, 100000, 2, 40), (4, 9000, 1, 64), (3, 4096, 1, 40),
    (3, 2, 3, 40), (2, 70001, 1, 64)])
def test_sort_random_words(words, n, arrays, top):
    rng = np.random.default_rng(1000 + 7 * words + n % 97)
    say(f"sort: {arrays} x {n} pairs, {words} words, top word {top} bits")
    _run(_keys(rng, arrays, words, n, top), _ids(arrays, n))


def test_sort_one_varying_word_of_three():
    # words 0 and 2 constant within each array (different per array): the
    # single-word path on a three-word key
    rng = np.random.default_rng(1011)
    arrays, n = 3, 30000
    k = np.empty((arrays, 3, n), dtype=np.uint64)
    for a in range(arrays):
        k[a, 0, :] = np.uint64(rng.integers(0, 2**40))
        k[a, 2, :] = np.uint64(rng.integers(0, 2**63))
    k[:, 1, :] = rng.integers(0, 2**63, size=(arrays, n), dtype=np.uint64)
    _run(k, _ids(arrays, n))


def test_sort_duplicates_keep_input_order():
    # few distinct keys, ids in a shuffled order: equal keys must keep it
    rng = np.random.default_rng(1012)
    arrays, n = 2, 50000
    pool = _keys(rng, 1, 2, 37, 64)[0]
    pick = rng.integers(0, 37, size=(arrays, n))
    k = np.stack([pool[:, pick[a]] for a in range(arrays)])
    _run(k, _ids(arrays, n, ascending=False, rng=rng))


def test_sort_constant_digits_skipped():
    # values below 2^20 in one word: most digit positions never vary
    rng = np.random.default_rng(1013)
    k = rng.integers(0, 1 << 20, size=(2, 1, 20000), dtype=np.uint64)
    _run(k, _ids(2, 20000))


def test_sort_all_equal_keys():
    k = np.full((2, 3, 5000), np.uint64(0x1234), dtype=np.uint64)
    rng = np.random.default_rng(1014)
    _run(k, _ids(2, 5000, ascending=False, rng=rng))
