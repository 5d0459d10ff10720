"""Pins of the sort oracle against brute force, invariants and closed forms.

The oracle is the plain definition of sort / sortperm / segmented sort
(paper Sec. II-B, with Julia Base ordering).  These tests check it against
things other than itself: a separately written insertion sort and
comparator, exhaustive permutations, closed forms, and invariants that are
shown to reject planted mistakes.
"""
import itertools
import os
import zlib

import numpy as np
import pytest

import oracle
from oracle import brute
from oracle.rmi import key_image
from pools import DTYPES, NP, bits, random_keys, special_bits


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("kind", ["mixed", "ties", "uniform"])
def test_sortperm_matches_insertion_sort(dt, kind):
    rng = np.random.default_rng(zlib.crc32(f"{dt}{kind}".encode()))
    for n in [0, 1, 2, 3, 7, 64, 257]:
        k = random_keys(dt, n, rng, kind)
        assert np.array_equal(oracle.sortperm(k), brute.insertion_sortperm(k)), (dt, kind, n)


@pytest.mark.parametrize("dt", DTYPES)
def test_sort_matches_insertion_sort_bitwise(dt):
    rng = np.random.default_rng(7)
    for n in [0, 1, 5, 100, 300]:
        k = random_keys(dt, n, rng, "mixed")
        assert np.array_equal(bits(oracle.sort(k)), bits(brute.insertion_sort(k)))


@pytest.mark.parametrize("dt", ["f32", "f64", "i32", "u64"])
def test_exhaustive_permutations_small(dt):
    """Every ordering of a 6-element multiset of specials sorts to the same
    bits (except NaN order, which must follow input order)."""
    sp = special_bits(dt)
    rng = np.random.default_rng(3)
    base = sp[rng.choice(sp.size, size=6, replace=True)]
    expect = None
    for p in itertools.permutations(range(6)):
        k = base[list(p)]
        perm = oracle.sortperm(k)
        assert np.array_equal(perm, brute.insertion_sortperm(k))
        out = oracle.sort(k)
        assert np.array_equal(bits(out), bits(k[perm]))
        if dt.startswith("f"):
            nn = out[~np.isnan(out)]
            if expect is None:
                expect = bits(nn).copy()
            assert np.array_equal(bits(nn), expect)
            # NaNs appear last, in input order
            nan_in = bits(k[np.isnan(k)])
            assert np.array_equal(bits(out[out.size - nan_in.size:]), nan_in)


def test_float_order_closed_form():
    """Shuffles of the golden float32 order sort back to it."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "float32_total_order.txt")
    vals = [int(l.split()[0], 16) for l in open(path) if l.strip() and not l.startswith("#")]
    order = np.array(vals, dtype=np.uint32)
    rng = np.random.default_rng(11)
    for _ in range(20):
        shuf = rng.permutation(order)
        assert np.array_equal(bits(oracle.sort(shuf.view(np.float32))), order)


@pytest.mark.parametrize("dt", DTYPES)
def test_closed_forms(dt):
    rng = np.random.default_rng(5)
    n = 5000
    # a permutation of distinct values sorts to the ascending sequence, and
    # sortperm of a permutation is its inverse
    if dt.startswith("f"):
        base = np.arange(n, dtype=NP[dt]) - n / 2
    else:
        base = (np.arange(n) + (np.iinfo(NP[dt]).min // 2 if dt[0] == "i" else 0)).astype(NP[dt])
    p = rng.permutation(n)
    k = base[p]
    assert np.array_equal(oracle.sort(k), base)
    inv = np.empty(n, dtype=np.int64)
    inv[p] = np.arange(n)
    assert np.array_equal(oracle.sortperm(k).astype(np.int64), inv)
    # constant array: unchanged, perm = iota
    c = np.full(n, base[17], dtype=NP[dt])
    assert np.array_equal(oracle.sortperm(c), np.arange(n, dtype=np.uint32))
    # reverse-sorted distinct values
    assert np.array_equal(oracle.sortperm(base[::-1].copy()).astype(np.int64), np.arange(n)[::-1])


@pytest.mark.parametrize("dt", DTYPES)
def test_invariants_and_planted_mistakes(dt):
    rng = np.random.default_rng(9)
    k = random_keys(dt, 400, rng, "mixed")
    out = oracle.sort(k)
    perm = oracle.sortperm(k)
    assert brute.is_nondecreasing(out)
    assert brute.same_multiset(out, k)
    assert brute.perm_is_stable_sort(k, perm)
    assert np.array_equal(bits(k[perm]), bits(out))
    # planted mistakes must be caught by the checkers
    i = int(np.argmax(out != out[0]))            # an index with a larger key
    swapped = out.copy()
    swapped[[0, i]] = swapped[[i, 0]]
    if brute.isless(out[0].item(), out[i].item()):
        assert not brute.is_nondecreasing(swapped)
    dropped = out.copy()
    dropped[1] = dropped[2] if not np.array_equal(bits(dropped[1:2]), bits(dropped[2:3])) else dropped[1]
    if not np.array_equal(bits(dropped), bits(out)):
        assert not brute.same_multiset(dropped, k)
    # an unstable tie: swap two equal keys in the permutation
    _, first = np.unique(bits(k[perm]), return_index=True)
    vals, counts = np.unique(bits(k), return_counts=True)
    dup = vals[counts > 1]
    if dup.size:
        pos = np.nonzero(bits(k[perm]) == dup[0])[0]
        bad = perm.copy()
        bad[[pos[0], pos[1]]] = bad[[pos[1], pos[0]]]
        assert not brute.perm_is_stable_sort(k, bad)


@pytest.mark.parametrize("dt", DTYPES)
def test_key_image_orders_like_comparator(dt):
    """A stable sort keyed on the oracle's order-preserving unsigned image
    gives the comparator sort's permutation (special patterns + random bits)."""
    rng = np.random.default_rng(13)
    k = np.concatenate([special_bits(dt), random_keys(dt, 3000, rng, "mixed")])
    by_image = np.argsort(key_image(k), kind="stable").astype(np.uint32)
    assert np.array_equal(by_image, oracle.sortperm(k))


@pytest.mark.parametrize("threads", [1, 2, 3, 8, 13])
def test_sort_mt_equals_sort(threads):
    rng = np.random.default_rng(threads)
    for dt in ["f32", "i64", "u64", "f64"]:
        k = random_keys(dt, 20011, rng, "mixed")
        assert np.array_equal(bits(oracle.sort_mt(k, threads)), bits(oracle.sort(k)))


def test_segsort():
    rng = np.random.default_rng(21)
    k = random_keys("f32", 3000, rng, "mixed")
    cuts = np.sort(rng.integers(0, 3000, size=40))
    off = np.concatenate([[0], cuts, [3000], [3000]]).astype(np.int64)   # incl. empties
    out = oracle.segsort(k, off)
    for s in range(off.size - 1):
        a, b = off[s], off[s + 1]
        assert np.array_equal(bits(out[a:b]), bits(brute.insertion_sort(k[a:b])))
    # keys outside [off[0], off[-1]) are untouched
    off2 = np.array([100, 200, 2500], dtype=np.int64)
    out2 = oracle.segsort(k, off2)
    assert np.array_equal(bits(out2[:100]), bits(k[:100]))
    assert np.array_equal(bits(out2[2500:]), bits(k[2500:]))
    # one segment == sort
    assert np.array_equal(bits(oracle.segsort(k, np.array([0, 3000]))), bits(oracle.sort(k)))


@pytest.mark.parametrize("dt", DTYPES)
def test_searchsorted_matches_counting(dt):
    """Sec. II-B searchsortedfirst / searchsortedlast: the oracle's bisection
    against counting with the separately written comparator, on sorted
    haystacks with repeats and (floats) NaNs, signed zeros and infinities;
    needles are haystack members, specials and random keys."""
    rng = np.random.default_rng(zlib.crc32(f"search{dt}".encode()))
    for n in [0, 1, 2, 9, 64, 301]:
        v = oracle.sort(random_keys(dt, n, rng, "ties" if n % 2 else "mixed"))
        x = np.concatenate([v[rng.integers(0, max(n, 1), size=min(n, 40))] if n else v,
                            special_bits(dt).view(NP[dt]), random_keys(dt, 40, rng, "mixed")])
        for last in (False, True):
            got = oracle.searchsorted(v, x, last)
            assert np.array_equal(got, brute.count_search(v, x, last)), (dt, n, last)


def test_searchsorted_closed_forms():
    """Worked cases: repeats give the ends of their run; below every element
    gives 0 / -1; above every element gives n / n-1; -0.0 sits before +0.0
    and NaN after +inf (all NaNs tie)."""
    v = np.array([1, 3, 3, 3, 7, 9], dtype=np.int64)
    x = np.array([0, 1, 2, 3, 4, 9, 10], dtype=np.int64)
    assert oracle.searchsorted(v, x, False).tolist() == [0, 0, 1, 1, 4, 5, 6]
    assert oracle.searchsorted(v, x, True).tolist() == [-1, 0, 0, 3, 3, 5, 5]
    f = np.array([-np.inf, -0.0, 0.0, 0.0, np.inf, np.nan, np.nan], dtype=np.float64)
    q = np.array([-0.0, 0.0, np.nan, np.inf, 5.0], dtype=np.float64)
    assert oracle.searchsorted(f, q, False).tolist() == [1, 2, 5, 4, 4]
    assert oracle.searchsorted(f, q, True).tolist() == [1, 3, 6, 4, 3]
    # the empty haystack
    e = np.array([], dtype=np.float32)
    assert oracle.searchsorted(e, np.array([1.0], np.float32), False).tolist() == [0]
    assert oracle.searchsorted(e, np.array([1.0], np.float32), True).tolist() == [-1]


def test_searchsorted_planted_mistake_is_caught():
    """An off-by-one in the bisection (using <= for the first-index search)
    differs from counting on a haystack with repeats."""
    v = np.array([2, 2, 5], dtype=np.int32)
    x = np.array([2], dtype=np.int32)
    wrong_first = oracle.searchsorted(v, x, True) + 1   # upper bound instead of lower bound
    assert not np.array_equal(wrong_first, brute.count_search(v, x, False))


@pytest.mark.parametrize("dt", ["i32", "i64", "u32", "u64"])
def test_accumulate_integers_match_big_int_sums(dt):
    """Sec. II-B accumulate with +: the oracle against Python's unbounded
    integers reduced modulo 2^width (wrap-around), inclusive and exclusive."""
    rng = np.random.default_rng(zlib.crc32(f"acc{dt}".encode()))
    w = 32 if dt.endswith("32") else 64
    for n in [0, 1, 2, 17, 1000]:
        x = random_keys(dt, n, rng, "uniform")
        run, inc, exc = 0, [], []
        for v in x.tolist():
            exc.append(run)
            run += int(v)
            inc.append(run)
        for inclusive, ref in ((True, inc), (False, exc)):
            want = np.array([r % (1 << w) for r in ref], dtype=np.uint64 if w == 64 else np.uint32)
            got = oracle.accumulate(x, inclusive)
            assert np.array_equal(got.view(want.dtype), want), (dt, n, inclusive)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_accumulate_floats_match_exactly_rounded_sums(dt):
    """Float prefixes against math.fsum (the correctly rounded sum) of each
    prefix: equal to within a few units of float64 rounding."""
    import math
    rng = np.random.default_rng(zlib.crc32(f"accf{dt}".encode()))
    x = (rng.standard_normal(600) * np.exp(rng.uniform(-20, 20, 600))).astype(NP[dt])
    inc = oracle.accumulate(x, True)
    exc = oracle.accumulate(x, False)
    xs = [float(v) for v in x]
    for i in range(x.size):
        s_inc = math.fsum(xs[: i + 1])
        s_exc = math.fsum(xs[:i])
        scale = math.fsum(abs(v) for v in xs[: i + 1])
        assert abs(inc[i] - s_inc) <= 4e-16 * scale + 1e-300
        assert abs(exc[i] - s_exc) <= 4e-16 * scale + 1e-300


def test_accumulate_closed_forms():
    """All ones: i + 1 inclusive, i exclusive; 0..n-1: the Gauss sums; a
    planted shift (exclusive read as inclusive) is caught."""
    n = 5000
    ones = np.ones(n, dtype=np.int64)
    assert np.array_equal(oracle.accumulate(ones, True), np.arange(1, n + 1))
    assert np.array_equal(oracle.accumulate(ones, False), np.arange(n))
    r = np.arange(n, dtype=np.uint64)
    i = np.arange(n, dtype=np.uint64)
    assert np.array_equal(oracle.accumulate(r, True), i * (i + np.uint64(1)) // np.uint64(2))
    assert np.array_equal(oracle.accumulate(r, False), i * (i - np.uint64(1)) // np.uint64(2) * (i > 0))
    f = np.full(n, 0.5, dtype=np.float32)
    assert np.array_equal(oracle.accumulate(f, True), 0.5 * np.arange(1, n + 1))
    assert not np.array_equal(oracle.accumulate(ones, False), oracle.accumulate(ones, True))
    # wrap-around: int32 max + 1 wraps to int32 min
    w = np.array([2**31 - 1, 1], dtype=np.int32)
    assert oracle.accumulate(w, True).tolist() == [2**31 - 1, -(2**31)]


# ------------------------------------------- 16- and 128-bit integer keys
from pools import WIDE_DTYPES, rows128, special128, wide_arg, wide_keys  # noqa: E402


@pytest.mark.parametrize("dt", WIDE_DTYPES)
@pytest.mark.parametrize("kind", ["mixed", "ties", "uniform"])
def test_wide_sortperm_matches_insertion_sort(dt, kind):
    rng = np.random.default_rng(zlib.crc32(f"{dt}{kind}".encode()))
    wd = wide_arg(dt)
    for n in [0, 1, 2, 3, 7, 64, 301]:
        k = wide_keys(dt, n, rng, kind)
        perm = oracle.sortperm(k, wd)
        assert np.array_equal(perm, brute.insertion_sortperm(k, wd)), (dt, kind, n)
        assert np.array_equal(oracle.sort(k, wd), k[perm.astype(np.int64)]), (dt, kind, n)


@pytest.mark.parametrize("dt", ["i16", "i128", "u128"])
def test_wide_exhaustive_permutations_small(dt):
    rng = np.random.default_rng(13)
    wd = wide_arg(dt)
    sp = wide_keys(dt, 40, rng, "ties")
    base = sp[rng.choice(sp.shape[0], size=6, replace=True)]
    expect = None
    for p in itertools.permutations(range(6)):
        k = base[list(p)]
        perm = oracle.sortperm(k, wd)
        assert np.array_equal(perm, brute.insertion_sortperm(k, wd))
        out = oracle.sort(k, wd)
        expect = out if expect is None else expect
        assert np.array_equal(out, expect)


def test_int128_closed_forms():
    """Distinct values in a known order sort back to it; sortperm of a
    permutation is its inverse; the high word decides before the low word
    and the sign bit makes negatives smallest (signed) or largest
    (unsigned)."""
    rng = np.random.default_rng(17)
    ordered = [-(1 << 127), -(1 << 64) - 1, -(1 << 64), -2, -1, 0, 1, M := (1 << 64) - 1, M + 1,
               (5 << 64) | ((1 << 63) - 1), (5 << 64) | (1 << 63), (1 << 127) - 1]
    rows = rows128(ordered)
    for _ in range(10):
        p = rng.permutation(len(ordered))
        assert np.array_equal(oracle.sort(rows[p], "i128"), rows)
        assert np.array_equal(oracle.sortperm(rows[p], "i128"), np.argsort(p).astype(np.uint32))
    # unsigned: the same bit patterns, negatives now above every positive
    uo = sorted(v & ((1 << 128) - 1) for v in ordered)
    assert np.array_equal(oracle.sort(rows[rng.permutation(len(ordered))], "u128"), rows128(uo))
    # a larger closed form: a shuffled progression with a step above 2**64
    vals = [i * ((1 << 64) + 3) - (1 << 100) for i in range(3000)]
    r = rows128(vals)
    p = rng.permutation(len(vals))
    assert np.array_equal(oracle.sort(r[p], "i128"), r)


def test_int16_closed_forms():
    rng = np.random.default_rng(19)
    a = np.arange(-32768, 32768, dtype=np.int64).astype(np.int16)
    p = rng.permutation(a.size)
    assert np.array_equal(oracle.sort(a[p]), a)
    assert np.array_equal(oracle.sortperm(a[p]), np.argsort(p).astype(np.uint32))
    u = a.view(np.uint16)                        # every 16-bit pattern once
    assert np.array_equal(oracle.sort(u[p]), np.arange(65536).astype(np.uint16))


def test_int128_planted_mistake_is_caught():
    """Sorting 128-bit keys by their low word only (a plausible slip) or as
    unsigned when they are signed differs from the oracle on the pools."""
    rng = np.random.default_rng(23)
    k = wide_keys("i128", 200, rng, "mixed")
    ref = oracle.sort(k, "i128")
    assert not np.array_equal(k[np.argsort(k[:, 0], kind="stable")], ref)
    assert not np.array_equal(oracle.sort(k, "u128"), ref)


def test_sort_by_key_definition():
    """Payloads travel with their keys: an index payload reproduces the
    stable sortperm; equal keys keep their payloads in input order; keys and
    payloads match the brute-force permutation for every key dtype."""
    rng = np.random.default_rng(29)
    for dt in DTYPES + WIDE_DTYPES:
        wd = wide_arg(dt)
        k = wide_keys(dt, 500, rng, "ties") if dt in WIDE_DTYPES else random_keys(dt, 500, rng, "ties")
        idx = np.arange(500, dtype=np.uint32)
        ks, vs = oracle.sort_by_key(k, idx, wd)
        bp = brute.insertion_sortperm(k, wd)
        assert np.array_equal(vs, bp), dt
        assert np.array_equal(ks.view(np.uint8), k[bp.astype(np.int64)].view(np.uint8)), dt
        pay = rng.integers(0, 1 << 64, size=500, dtype=np.uint64)
        _, vs2 = oracle.sort_by_key(k, pay, wd)
        assert np.array_equal(vs2, pay[bp.astype(np.int64)]), dt
