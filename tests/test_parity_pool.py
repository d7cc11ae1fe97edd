"""The process pool that runs the oracle's search for the large parity
tests returns what one direct oracle call returns (CPU only)."""
import numpy as np
import pytest

import oracle as O
import synth
from tests.parity import OraclePool


@pytest.fixture(scope="module")
def pool():
    p = OraclePool(2)
    yield p
    p.close()


@pytest.mark.parametrize("mode,k,s", [("exhaustive", 3, 4), ("fast", 3, 4), ("gnu", 3, 4), ("exhaustive", 5, 3),
                                      ("fast", 5, 8)])
def test_pool_equals_one_call(pool, mode, k, s):
    I = synth.voronoi(97, 131, n_cells=40, n_dots=12, dot_px=(1, 3), seed=k * 10 + s).astype(np.float16)
    L = O.downsample_point(I, s)
    rng = np.random.default_rng(5)
    for pix in (None, np.sort(rng.choice(97 * 131, 3000, replace=False)), np.arange(0)):
        ref = O.search(I, L, s, k, 1e-3, mode, pixels=pix) if pix is None or pix.size else None
        got = pool.search(I, L, s, k, 1e-3, mode, pixels=pix, chunk=500)
        if ref is None:
            assert got.a.size == 0
            continue
        for f in ("a", "b", "alpha", "err"):
            assert np.array_equal(getattr(got, f), getattr(ref, f)), f
