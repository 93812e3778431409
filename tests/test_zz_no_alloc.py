"""bem_matvec_noalloc (the product that allocates nothing, for callers that cannot call hipMalloc)
against bem_matvec, through the C-ABI.

The two entry points run the same kernels in the same order, so their outputs must be bit-identical.
Calls in a row on one device share the static scratch array: a larger product first, then smaller
ones (fewer columns, a smaller matrix, the one-block plain path), each checked; a product whose
scratch need exceeds the array is refused with BEM_E_INVALID_ARG while the FP32 product of the same
matrix (half the scratch) runs.
"""
import numpy as np
import pytest

from paper_2310_09204_amd import lib, meshes

pytestmark = pytest.mark.gpu


def _noalloc(p, x, fp32):
    dx = lib.DeviceArray(x)
    dy = lib.DeviceArray(shape=x.shape)
    try:
        p.matvec_noalloc(dx.ptr, x.shape[0], dy.ptr, fp32=fp32)
        return dy.get()
    finally:
        dx.close()
        dy.close()


@pytest.fixture(scope="module")
def problems(ctx):
    big = meshes.crossed(24)
    small = meshes.unit_square(16)
    tiny = meshes.unit_square(8)
    out = [lib.Problem(ctx, m.vertices, m.triangles, precision=lib.FP32_REFINE) for m in (big, small, tiny)]
    yield out
    for p in out:
        p.close()


def test_noalloc_matches_matvec_in_a_row(problems):
    big, small, tiny = problems
    print("case noalloc: N = %d, %d, %d" % (big.N, small.N, tiny.N), flush=True)
    rng = np.random.default_rng(1)
    for p, k in ((big, 17), (big, 16), (small, 3), (tiny, 2), (small, 1)):
        x = rng.standard_normal((k, p.N))
        for fp32 in (False, True):
            y_ref = p.matvec(x, fp32=fp32)
            y = _noalloc(p, x, fp32)
            assert y.shape == y_ref.shape
            assert np.array_equal(y, y_ref), (p.N, k, fp32, np.abs(y - y_ref).max())


def test_noalloc_refuses_a_product_beyond_its_scratch(ctx):
    # crossed panels at h = 1/80: N = 18,961 > 16,128, the FP64 limit; the FP32 product fits
    m = meshes.crossed(80)
    p = lib.Problem(ctx, m.vertices, m.triangles, precision=lib.FP32_REFINE)
    try:
        print("case noalloc limit: N = %d" % p.N, flush=True)
        assert 16128 < p.N <= 32256
        x = np.random.default_rng(2).standard_normal((2, p.N))
        with pytest.raises(lib.BemError) as e:
            _noalloc(p, x, fp32=False)
        assert e.value.code == -1 and "scratch" in str(e.value)
        assert np.array_equal(_noalloc(p, x, fp32=True), p.matvec(x, fp32=True))
    finally:
        p.close()
        ctx.release_cached()
