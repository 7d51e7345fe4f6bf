"""GPU parity of the energy-partition model of Sec. III.B (hyb_model_scan)
against the FP64 oracle, and its properties over the paper's intensity-Z
plane."""
import numpy as np
import pytest

import workloads as W
from oracle import model as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_01723_amd as P
    P.check_abi()
    return P


def test_model_scan_matches_oracle(P):
    """56 points (7 intensities x 8 elements, 1000 steps): every fraction
    within 1e-10 of the oracle's (the same integration in FP64)."""
    m = W.model_inputs(nsteps=1000)
    I, Z = W.model_scan_grid(n_int=7, z_values=[1, 4, 13, 29, 47, 74, 79, 92])
    got = P.model_scan(m, I, Z)
    ref = M.partition(m, I, Z, m["nsteps"])
    err = np.max(np.abs(got - ref))
    print(f"  max |GPU - oracle| over {got.size} fractions: {err:.2e}", flush=True)
    assert err < 1e-10


def test_model_plane_properties(P):
    """The paper's plane (41 intensities over 1e20-1e22 W/cm^2 x Z = 1..92,
    4000 steps): energy conserved at every point, 24 sampled points equal to
    the oracle's, and the dominant mechanisms of Sec. III.B."""
    m = W.model_inputs()
    I, Z = W.model_scan_grid()
    got = P.model_scan(m, I, Z)
    assert got.shape == (6, len(I))
    assert np.allclose(got[0] + got[2] + got[3] + got[4] + got[5], 1.0, rtol=0, atol=1e-9)
    pick = np.random.default_rng(2).choice(len(I), 24, replace=False)
    ref = M.partition(m, I[pick], Z[pick], m["nsteps"])
    assert np.max(np.abs(got[:, pick] - ref)) < 1e-10
    k = lambda i0, z: int(np.nonzero((np.isclose(I, W.intensity_wcm2(i0))) & (Z == z))[0][0])
    names = ("brem", "ionisation", "reflux", "field", "escaped")
    dom = [names[int(np.argmax(got[[0, 2, 3, 4, 5], k(i0, z)]))] for i0, z in ((1e20, 79), (1e22, 79), (1e22, 13))]
    assert dom == ["ionisation", "brem", "reflux"]
    eta = got[1].reshape(41, 92)
    print(f"  eta_e->gamma: Al 1e20 {eta[0, 12]:.4f}, Au 1e22 {eta[-1, 78]:.4f}", flush=True)
    assert np.all(np.diff(eta[:, 78]) > 0)            # Au: rises with intensity


def test_model_rejects_bad_inputs(P):
    m = W.model_inputs(nsteps=10)
    with pytest.raises(P.HybError):
        P.model_scan(m, [1e24], [0.5])
    with pytest.raises(P.HybError):
        P.model_scan(dict(m, nsteps=0), [1e24], [13.0])
    assert P.model_scan(m, [], []).shape == (6, 0)
