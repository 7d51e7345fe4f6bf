"""GPU parity of the hot-current deposit (eq. Ampere_Maxwell's j_h, App. A)
and the collisional heat on dense states, where every workgroup of the
particle kernel runs several chunks: the LDS regions carried from chunk to
chunk, the third region of FP32-mixed runs and the deposits outside the
chunk's homes all meet the oracle, node by node.

States go in through hyb_set_state in tile order (4^3-cell tiles, x fastest),
as the sort leaves them; the oracle steps the same state (in FP32-mixed runs
the state as the GPU stores it, read back) and its j_h, collisional heat,
fields, temperatures and resistivity after the step are compared with the
GPU's over the whole grid."""
import numpy as np
import pytest

import workloads as W
from oracle import OracleRun

from parity_util import field_rel, rel

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

MEC = 9.1093837015e-31 * 299792458.0


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_01723_amd as P
    P.check_abi()
    return P


def _cfg(precision, n):
    cfg = W.base_config(nx=64, ny=32, nz=32, dx=1e-6, dt=20e-15, precision=precision,
                        x_lo=0.0, x_hi=64e-6, I0=W.intensity_wcm2(1e21), sort_every=1,
                        max_particles=n, series_len=4, tally_nE=16, tally_ntheta=18)
    return cfg


def _tile_order(cells, cfg):
    ntx, nty = cfg["nx"] // 4, cfg["ny"] // 4
    t = (cells[:, 0] >> 2) + ntx * ((cells[:, 1] >> 2) + nty * (cells[:, 2] >> 2))
    return np.argsort(t, kind="stable")


def _state(pos, p, w, rng, cfg):
    n = len(w)
    cells = np.floor(pos / cfg["dx"]).astype(np.int64)
    o = _tile_order(cells, cfg)
    return dict(pos=pos[o], p=p[o], w=w[o], tau=-np.log(1.0 - rng.uniform(size=n))[o] + 0.5,
                ids=np.arange(n, dtype=np.uint32)[o], step=10, next_id=n)


def _run_both(P, cfg, st):
    """The GPU steps st once; the oracle steps the state the GPU holds."""
    run = P.Run(cfg)
    run.set_state(st)
    st_gpu = run.get_state()
    run.step(1)
    got = run.get_state()
    run.close()
    ora = OracleRun(cfg)
    ora.set_state(dict(st_gpu, step=st["step"], next_id=st["next_id"]))
    ora.step()
    return got, ora.state()


def _compare_grid(got, ref, tol_j, tol_heat, tol_field):
    ej = field_rel(got["j"], ref["j"])
    eh = rel(got["ion_heat"], ref["ion_heat"])
    eE, eB = field_rel(got["E"], ref["E"]), field_rel(got["B"], ref["B"])
    eT = rel(got["Te"], ref["Te"])
    eeta = rel(got["eta"], ref["eta"])
    print(f"  j {ej:.2e} heat {eh:.2e} E {eE:.2e} B {eB:.2e} Te {eT:.2e} eta {eeta:.2e}", flush=True)
    assert ej <= tol_j
    assert eh <= tol_heat
    assert eE <= tol_field and eB <= tol_field
    assert eT <= tol_field and eeta <= tol_field


@pytest.mark.parametrize("precision", [W.FP64, W.FP32_MIXED])
def test_deposit_one_cell_worst_case(P, precision):
    """2.2e6 electrons of one weight in one cell, all on the node of their x
    edge and moving along +x at gamma ~ 10: every contribution to that
    node's j_x is near the largest a contribution can be (2^23 FP32 units),
    and a workgroup's carried region sums three chunks of them, 384 per
    word, before its flush -- past 2^31, where 32-bit words wrapped."""
    n = 2_200_000
    cfg = _cfg(precision, n)
    rng = np.random.default_rng(3)
    c = np.array([21, 13, 17])
    pos = np.tile((c + np.array([0.5, 1e-3, 1e-3])) * cfg["dx"], (n, 1))
    p = np.zeros((n, 3))
    p[:, 0] = MEC * rng.uniform(9.0, 11.0, n)
    w = np.full(n, 1e3)
    got, ref = _run_both(P, cfg, _state(pos, p, w, rng, cfg))
    jmax = np.max(np.abs(ref["j"][0]))
    print(f"  max |j_x| {jmax:.3e} A/m^2", flush=True)
    assert jmax > 0
    tol = 1e-10 if precision == W.FP64 else 1e-5
    _compare_grid(got, ref, tol, 1e-10 if precision == W.FP64 else 1e-4, 1e-10 if precision == W.FP64 else 1e-5)


@pytest.mark.parametrize("precision", [W.FP64, W.FP32_MIXED])
def test_deposit_dense_uneven_tiles(P, precision):
    """~2.6e6 electrons in tiles of very uneven population (a row of tiles
    holding 50 to 1.2e6 electrons, and scattered thin tiles), random
    directions and exponential energies: chunks that span several tiles,
    homes carried over many chunks, thin tiles outside the homes."""
    rng = np.random.default_rng(5)
    row = [(2, 3, 3, 5000), (3, 3, 3, 40), (4, 3, 3, 1_200_000), (5, 3, 3, 150), (6, 3, 3, 900_000),
           (7, 3, 3, 60), (8, 3, 3, 300_000), (9, 3, 3, 7)]
    extra = [(int(rng.integers(1, 15)), int(rng.integers(1, 7)), int(rng.integers(1, 7)),
              int(rng.integers(1, 3000))) for _ in range(60)]
    pos, p, w = [], [], []
    for tx, ty, tz, k in row + extra:
        lo = np.array([tx, ty, tz]) * 4
        x = (lo + rng.uniform(0, 4, size=(k, 3))) * 1e-6
        e = rng.exponential(3.0, k) + 0.05                    # MeV
        g = 1 + e / 0.51099895
        um = np.sqrt(g * g - 1)
        d = rng.normal(size=(k, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        pos.append(x)
        p.append(MEC * um[:, None] * d)
        w.append(rng.uniform(0.6e3, 1.0e3, k))
    pos, p, w = np.vstack(pos), np.vstack(p), np.concatenate(w)
    n = len(w)
    cfg = _cfg(precision, n)
    got, ref = _run_both(P, cfg, _state(pos, p, w, rng, cfg))
    fp64 = precision == W.FP64
    _compare_grid(got, ref, 1e-10 if fp64 else 1e-5, 1e-10 if fp64 else 1e-4, 1e-10 if fp64 else 1e-5)
