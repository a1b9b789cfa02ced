"""MFMA GEMM kernels (FP64, FP32, split-BF16) against numpy, all tiles and operand layouts.

Long-K shapes with a tiny output take the deterministic split-K path.

Ragged shapes exercise the bounds of every tile; shapes whose leading dimensions are
multiples of 4 run the 16-byte vector-load kernels (multiples of 8 for split-BF16).  Errors are measured
against sum_k |alpha a_ik b_kj| + |beta c_ij| (the scale of the rounding
bound of each dot product): FP64 1e-13, FP32 1e-5, split-BF16 1e-4.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-13, "fp32": 1e-5, "bf16x3": 1e-4}


@pytest.fixture(scope="module")
def ctx():
    import paper_2509_14157_amd as P
    with P.Context(0) as c:
        yield c


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_gemm_all_tiles_and_layouts(ctx, prec):
    rng = np.random.default_rng(1)
    bad = []
    for tile in range(17):  # every tile: 6 single-, 5 double-buffered, 256x64, 64x256, two with k depth 32, two FP32-only
        # (16, 16, 4), (132, 68, 40) and (260, 196, 36) have every leading dimension a
        # multiple of 4: they take the 16-byte vector loads, with ragged M, N and K edges;
        # the last three have every leading dimension a multiple of 8, which the
        # split-BF16 vector staging needs (ragged edges of 8, split-K with aligned slices)
        for (M, N, K) in ((37, 53, 29), (130, 70, 45), (16, 16, 4), (1, 70, 33), (257, 129, 3),
                          (3, 5, 5000), (1, 1, 70001), (132, 68, 40), (260, 196, 36),
                          (264, 136, 72), (40, 48, 1000), (8, 16, 4096)):
            for ak in (True, False):
                for bn in (True, False):
                    A = rng.normal(size=(M, K))
                    B = rng.normal(size=(K, N))
                    C = rng.normal(size=(M, N))
                    ref = 0.7 * A @ B + 0.3 * C
                    got = ctx.debug_gemm(A, B, C, alpha=0.7, beta=0.3, prec=prec, tile=tile, a_kfast=ak, b_nfast=bn)
                    # rounding bound of a dot product scales with sum_k |a_k b_k|
                    scale = (0.7 * np.abs(A) @ np.abs(B) + 0.3 * np.abs(C)).max()
                    err = np.abs(got - ref).max() / scale
                    if err > TOL[prec]:
                        bad.append((tile, M, N, K, ak, bn, err))
    assert not bad, bad


def test_gemm_empty_k_scales_c(ctx):
    C = np.arange(12.0).reshape(3, 4)
    got = ctx.debug_gemm(np.zeros((3, 0)), np.zeros((0, 4)), C, alpha=1.0, beta=2.0)
    assert np.array_equal(got, 2 * C)


@pytest.mark.parametrize("M", [192, 193, 207, 208, 209, 590])
def test_gemm_fp64_partial_last_m_tile(ctx, M):
    """FP64 128 x 128 vector tile on a partial last M tile: a wavefront whose sub-tile
    holds at most 16 rows of C runs the one-block loop (M = 192, 193, 207, 208, and 590:
    the ring's 78-row fifth tile), one with 17 runs every block (M = 209)."""
    rng = np.random.default_rng(M)
    N, K = 136, 40
    for bn in (True, False):
        A = rng.normal(size=(M, K))
        B = rng.normal(size=(K, N))
        C = rng.normal(size=(M, N))
        ref = 1.3 * A @ B - 0.5 * C
        got = ctx.debug_gemm(A, B, C, alpha=1.3, beta=-0.5, prec="fp64", tile=3, a_kfast=True, b_nfast=bn)
        scale = (1.3 * np.abs(A) @ np.abs(B) + 0.5 * np.abs(C)).max()
        assert np.abs(got - ref).max() / scale < TOL["fp64"], (M, bn)
