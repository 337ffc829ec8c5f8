"""The allocation-free entry point dpd_pair_noise_noalloc against
dpd_pair_noise (same kernel): bit-exact, on two calls in a row, the second
smaller, and the size limit."""
import numpy as np
import pytest

from paper_1804_06205_amd import dpd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dpd.lib()


def _triples(rng, m):
    ti = rng.integers(0, 2 ** 32, size=m, dtype=np.uint64).astype(np.uint32)
    tj = rng.integers(0, 2 ** 32, size=m, dtype=np.uint64).astype(np.uint32)
    s = rng.integers(0, 2 ** 32, size=m, dtype=np.uint64).astype(np.uint32)
    return ti, tj, s


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_matches_allocating_entry_point(precision):
    rng = np.random.default_rng(91)
    seed = 0xFEDCBA9876543210
    # Two calls in a row on the shared device array: the full size, then a
    # smaller one (the first call's tail must not leak into the second).
    for m in (2 ** 18, 777):
        ti, tj, s = _triples(rng, m)
        print(f"noalloc {precision} m={m}", flush=True)
        got = dpd.pair_noise_noalloc(seed, ti, tj, s, precision)
        ref = dpd.pair_noise(seed, ti, tj, s, precision)
        assert got.shape == (m,)
        np.testing.assert_array_equal(got, ref)


def test_noalloc_limits():
    rng = np.random.default_rng(92)
    ti, tj, s = _triples(rng, 2 ** 18 + 1)
    with pytest.raises(dpd.DPDError) as e:
        dpd.pair_noise_noalloc(1, ti, tj, s)
    assert e.value.code == dpd.EINVAL
    assert dpd.pair_noise_noalloc(1, ti[:0], tj[:0], s[:0]).shape == (0,)
