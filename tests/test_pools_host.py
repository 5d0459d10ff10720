"""Host checks of the shaped-input helpers the GPU tests use (no GPU)."""
import numpy as np
import pytest

import oracle
from pools import DTYPES, bits, from_image, prefix_groups


@pytest.mark.parametrize("w,t,n,long_group", [(32, 16, 4096, 0), (32, 16, 4096, 17), (64, 16, 16_384, 48),
                                              (32, 8, 256, 0), (64, 8, 200, 17)])
def test_prefix_groups_shape(w, t, n, long_group):
    rng = np.random.default_rng(1)
    a = prefix_groups(n, w, t, 16, rng, long_group)
    assert a.size == n and a.dtype == (np.uint32 if w == 32 else np.uint64)
    p = (a >> np.array(w - t, dtype=a.dtype)).astype(np.uint64)
    _, counts = np.unique(p, return_counts=True)
    if long_group:
        assert counts.max() == min(long_group, n) and np.sort(counts)[-2] <= 16
    else:
        assert counts.max() <= 16
    # the top bit and the lowest bit vary, and some group holds equal images
    assert p.min() == 0 and p.max() == (1 << t) - 1
    assert (a & 1).min() == 0 and (a & 1).max() == 1
    assert np.unique(a).size < a.size


@pytest.mark.parametrize("dt", DTYPES)
def test_from_image_keeps_the_order(dt):
    """Sorting the keys made from images (by the oracle's total order) puts
    them in the order of their images, ties aside (all NaNs tie)."""
    rng = np.random.default_rng(2)
    w = 32 if dt in ("i32", "u32", "f32") else 64
    img = rng.integers(0, 1 << min(w, 63), size=5000, dtype=np.uint64)
    if w == 64:
        img ^= rng.integers(0, 2, size=img.size, dtype=np.uint64) << np.uint64(63)
    img = img.astype(np.uint32 if w == 32 else np.uint64)
    k = from_image(img, dt)
    perm = oracle.sortperm(k)
    ordered = img[perm]
    if dt.startswith("f"):
        nan = np.isnan(k[perm])
        assert np.all(ordered[~nan][1:] >= ordered[~nan][:-1])
        assert nan.sum() == 0 or np.all(nan[np.argmax(nan):])      # NaNs last
    else:
        assert np.all(ordered[1:] >= ordered[:-1])
