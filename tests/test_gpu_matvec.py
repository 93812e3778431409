"""Products y = W x through the C-ABI: the symmetric upper-half product against a plain FP64
product of the same matrix, and a block of columns against the same columns one at a time, at sizes
that span several super-tiles with ragged last super-blocks and a ragged last 64-row block."""
import numpy as np
import pytest

from paper_2310_09204_amd import lib, meshes

pytestmark = pytest.mark.gpu

CASES = {
    # N = 1657: 26 blocks of 64 (last one 57 rows); super-blocks of 8 (FP32) and 4 (FP64) both ragged
    "crossed24": lambda: meshes.crossed(24),
    # N = 2209: 35 blocks (last one 33 rows)
    "square48": lambda: meshes.unit_square(48),
}


@pytest.fixture(scope="module", params=list(CASES))
def problem(request, ctx):
    m = CASES[request.param]()
    print("case matvec", request.param, m.nt, flush=True)
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=4, precision=lib.FP32_REFINE)
    yield request.param, p
    p.close()


@pytest.mark.parametrize("k", [1, 2, 5, 16, 17, 33])
def test_fp64_product(problem, k):
    name, p = problem
    W = p.matrix()
    assert np.array_equal(W, W.T)
    x = np.random.default_rng(10 + k).standard_normal((k, p.N))
    y = p.matvec(x)
    ref = x @ W
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err < 1e-13, (name, k, err)


def test_fp64_matches_single_columns(problem):
    name, p = problem
    x = np.random.default_rng(7).standard_normal((16, p.N))
    y = p.matvec(x)
    y1 = np.stack([p.matvec(x[c:c + 1])[0] for c in range(16)])
    err = np.abs(y - y1).max() / np.abs(y1).max()
    assert err < 1e-13, (name, err)


@pytest.mark.parametrize("k", [1, 2, 16, 19])
def test_fp32_product(problem, k):
    name, p = problem
    W32 = p.matrix().astype(np.float32).astype(np.float64)
    x = np.random.default_rng(20 + k).standard_normal((k, p.N))
    y = p.matvec(x, fp32=True)
    ref = x.astype(np.float32).astype(np.float64) @ W32
    # FP32 matrix-core sums over at most 512 products per partial, partials added in FP64
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err < 2e-6, (name, k, err)


def test_repeated_products_identical(problem):
    # fixed summation order: the same inputs give bit-identical outputs
    name, p = problem
    x = np.random.default_rng(3).standard_normal((16, p.N))
    for fp32 in (False, True):
        a = p.matvec(x, fp32=fp32)
        b = p.matvec(x, fp32=fp32)
        assert np.array_equal(a, b), (name, fp32)
