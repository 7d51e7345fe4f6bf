"""The allocation-free variant of the energy-partition model scan
(hyb_model_scan_static) against hyb_model_scan: the same kernel on the same
inputs, so the results must be identical; two calls in a row on the one GPU
array, the second with fewer points, and the size limit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_01723_amd as P
    P.check_abi()
    return P


def test_model_scan_static_equals_allocating_scan(P):
    from paper_2107_01723_amd import hyb
    m = W.model_inputs(nsteps=1000)
    I, Z = W.model_scan_grid(n_int=41)
    for sel in (slice(None), slice(5, 5 + 777)):     # 3772 points, then fewer
        i0, z = I[sel], Z[sel]
        want = hyb.model_scan(m, i0, z)
        got = hyb.model_scan_static(m, i0, z)
        print(f"  {len(i0)} points, max |diff| {np.max(np.abs(got - want)):.1e}", flush=True)
        assert got.shape == want.shape == (6, len(i0))
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, want)
    with pytest.raises(hyb.HybError) as e:
        hyb.model_scan_static(m, np.full(65537, 1e24), np.full(65537, 79.0))
    assert e.value.status == hyb.HYB_EINVAL
