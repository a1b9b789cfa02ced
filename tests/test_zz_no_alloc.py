"""The allocation-free fused triples entry point (fno_triples_residual_dev_noalloc)
against the allocating one, through the C ABI: two calls in a row, the second
on a smaller problem, each bit-identical to fno_triples_residual_dev on the
same inputs (same kernels; the static working array keeps the first call's
contents, which the second must not depend on); sizes beyond the array are
refused with FNO_ENOMEM before anything runs."""
import numpy as np
import pytest

from tests.helpers import HipBuffers
from tests.test_gpu_boundary import triples_dev_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2509_14157_amd as P
    return P


def test_noalloc_matches_allocating_entry_point(P):
    print("no-alloc triples residual: two calls, second smaller", flush=True)
    hip = HipBuffers()
    s = hip.stream()
    for (o, v, seed), prec in (((7, 24, 9), "fp64"), ((4, 12, 3), "fp64"), ((5, 14, 2), "fp32"),
                               ((6, 16, 4), "bf16x3")):
        arrays, _ = triples_dev_inputs(P, o, v, seed)
        ptrs = {k: hip.upload(x) for k, x in arrays.items()}
        n3 = arrays["T3"].size
        start = np.random.default_rng(seed).normal(0, 1, n3)  # R3 accumulates: start from nonzero values
        r_ref = hip.upload(start)
        r_got = hip.upload(start)
        P.triples_residual_dev(0, o, v, prec, ptrs, r_ref, s)
        P.triples_residual_dev(0, o, v, prec, ptrs, r_got, s, noalloc=True)
        hip.sync(s)
        ref, got = hip.download(r_ref, n3), hip.download(r_got, n3)
        assert np.array_equal(got, ref), (o, v, prec)
        assert np.abs(ref - start).max() > 0  # the call added the triples terms
    with pytest.raises(P.FnoError) as e:
        P.triples_residual_dev(0, 14, 64, "fp64", ptrs, r_got, s, noalloc=True)
    assert e.value.code == P.FNO_ENOMEM and "bytes" in str(e.value)
    hip.close(s)
