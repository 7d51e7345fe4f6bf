"""Pins of the grid-side oracle pieces that no closed form of the method
reached before: the Yee staggering of the gather (E on edges, B on faces,
App. A), the odd mirror ghosts at the walls, the edge resistivity of
eq. (Ohms_Law), the cell-centred |j_h|^2 of the Ohmic heating (App. A) and the
photon tally bins.

Each pin is a mathematical property, with positions taken from the Yee layout
as the grid description defines it (not from the oracle's tables):
  * trilinear interpolation reproduces a linear field exactly, so a gather at
    the right Yee positions returns the field's value at the particle;
  * a field odd about a wall (a product (x_d - wall) h(other axes)) is
    reproduced exactly up to the wall when the ghost one half-cell outside is
    minus the nearest value;
  * the mean of the four cells around an edge (or of the four edges around a
    cell centre) of a linear function is its value at the edge (centre);
  * photons placed at known bin centres and edges land in those bins.
Every pin is then shown to fail when a one-character mistake is planted in a
copy of the piece it guards (`test_pins_catch_planted_mistakes`)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import OracleRun
from oracle import fields as F
from oracle import particles as PT

# Yee positions (offset in cell units along x, y, z) from the grid layout:
#   Ex (i+1/2, j, k)  Ey (i, j+1/2, k)  Ez (i, j, k+1/2)
#   Bx (i, j+1/2, k+1/2)  By (i+1/2, j, k+1/2)  Bz (i+1/2, j+1/2, k)
YEE_E = ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5))
YEE_B = ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))
DIMS = (7, 5, 6)


def _coords(off, dims):
    """Coordinates (cell units) of the entries of one component array."""
    n1 = [d + 1 for d in dims]
    return np.meshgrid(*[np.arange(n1[d]) + off[d] for d in range(3)], indexing="ij")


def _valid(off, dims):
    """Entries inside the component's range (past a staggered range: unused)."""
    X = _coords(off, dims)
    return np.all([X[d] <= dims[d] for d in range(3)], axis=0)


def _linear(off, dims, a, b):
    X = _coords(off, dims)
    f = a + b[0] * X[0] + b[1] * X[1] + b[2] * X[2]
    return np.where(_valid(off, dims), f, 0.0)


def _interior_positions(rng, n, offs, dims):
    """Positions where every staggered axis of every component is at least a
    half cell from the walls (node axes span the whole grid)."""
    lo = np.zeros(3)
    hi = np.array(dims, dtype=float)
    for off in offs:
        for d in range(3):
            if off[d] == 0.5:
                lo[d] = 0.5
                hi[d] = dims[d] - 0.5
    return rng.uniform(lo, hi, size=(n, 3))


def check_gather_linear(gather=None, dims=DIMS, seed=11):
    """E and B built as linear functions at their Yee positions are gathered
    exactly at interior positions."""
    gather = gather or PT.gather
    rng = np.random.default_rng(seed)
    aE, bE = rng.normal(size=3), rng.normal(size=(3, 3))
    aB, bB = rng.normal(size=3), rng.normal(size=(3, 3))
    E = tuple(_linear(YEE_E[c], dims, aE[c], bE[c]) for c in range(3))
    B = tuple(_linear(YEE_B[c], dims, aB[c], bB[c]) for c in range(3))
    X = _interior_positions(rng, 400, YEE_E + YEE_B, dims)
    X = np.vstack([X, [[0.5, 0.5, 0.5], [dims[0] - 0.5, dims[1] - 0.5, dims[2] - 0.5]]])
    Ep, Bp = gather(X, E, B, dims)
    for c in range(3):
        assert np.allclose(Ep[:, c], aE[c] + X @ bE[c], rtol=0, atol=1e-12), f"E{c}"
        assert np.allclose(Bp[:, c], aB[c] + X @ bB[c], rtol=0, atol=1e-12), f"B{c}"


def check_gather_wall_ghosts(gather=None, dims=DIMS, seed=12):
    """For every component and each axis it is staggered along: a field odd
    about the lower (upper) wall, (x_d - wall) (1 + c . x_other), is gathered
    exactly within a half cell of that wall."""
    gather = gather or PT.gather
    rng = np.random.default_rng(seed)
    for fam, offs in (("E", YEE_E), ("B", YEE_B)):
        for c in range(3):
            for d in range(3):
                if offs[c][d] != 0.5:
                    continue
                for wall in (0.0, float(dims[d])):
                    cc = rng.normal(size=3)
                    cc[d] = 0.0
                    X0 = _coords(offs[c], dims)
                    f = (X0[d] - wall) * (1.0 + cc[0] * X0[0] + cc[1] * X0[1] + cc[2] * X0[2])
                    comp = np.where(_valid(offs[c], dims), f, 0.0)
                    zero = np.zeros_like(comp)
                    fields = [zero, zero, zero]
                    fields[c] = comp
                    # the other staggered axes of this component stay a half cell inside
                    X = _interior_positions(rng, 200, (offs[c],), dims)
                    X[:, d] = wall + (rng.uniform(0.0, 0.5, 200) if wall == 0.0 else -rng.uniform(1e-9, 0.5, 200))
                    Ep, Bp = gather(X, tuple(fields), tuple(fields), dims)
                    got = (Ep if fam == "E" else Bp)[:, c]
                    want = (X[:, d] - wall) * (1.0 + X @ cc)
                    assert np.allclose(got, want, rtol=0, atol=1e-12), f"{fam}{c} wall {wall} axis {d}"


def check_edge_eta(edge_eta=None, dims=DIMS, seed=13):
    """eta linear over the cell centres: interior edges carry its value at the
    edge centre; on a wall the clamped cells give the value at the nearest
    cell centre across it (zero gradient through the wall)."""
    edge_eta = edge_eta or F.edge_eta
    rng = np.random.default_rng(seed)
    a, b = 5.0, rng.normal(size=3)
    nx, ny, nz = dims
    C = np.meshgrid(*[np.arange(n) + 0.5 for n in dims], indexing="ij")
    eta = a + b[0] * C[0] + b[1] * C[1] + b[2] * C[2]
    got = edge_eta(eta)
    for c in range(3):
        X = _coords(YEE_E[c], dims)
        # the two transverse axes of the edge, clamped to the cell centres
        want = a + b[c] * X[c]
        for d in range(3):
            if d != c:
                want = want + b[d] * np.clip(X[d], 0.5, dims[d] - 0.5)
        ok = _valid(YEE_E[c], dims)
        assert np.allclose(got[c][ok], want[ok], rtol=0, atol=1e-12), f"edge family {c}"


def check_cell_current_sq(ccs=None, dims=DIMS, seed=14):
    """j_h linear at its edge positions: each cell-centred component is the
    linear value at the centre, so |j|^2 is exact."""
    ccs = ccs or F.cell_current_sq
    rng = np.random.default_rng(seed)
    a, b = rng.normal(size=3), rng.normal(size=(3, 3))
    j = tuple(_linear(YEE_E[c], dims, a[c], b[c]) for c in range(3))
    C = np.meshgrid(*[np.arange(n) + 0.5 for n in dims], indexing="ij")
    want = sum((a[c] + b[c][0] * C[0] + b[c][1] * C[1] + b[c][2] * C[2]) ** 2 for c in range(3))
    assert np.allclose(ccs(j), want, rtol=1e-12, atol=1e-12)


def _tally_run():
    cfg, _, _ = W.config_small()
    cfg.update(tally_nE=10, tally_ntheta=18, tally_Elo=1e4 * W.EV, tally_Ehi=1e9 * W.EV)
    return OracleRun(cfg)


def check_tally_bins(tally=None):
    """Photons at bin centres land in their bin; just above (below) an edge
    they land above (below) it; theta = pi is the last angle bin; below E_lo
    and at or above E_hi they go to the flow slots; the threshold sum and
    the step's series take k >= E_thr.  `tally(run, k, w, dirx, step)`."""
    tally = tally or OracleRun._tally
    r = _tally_run()
    nE, nth = r.hist_E.shape
    lo, hi = r.cfg["tally_Elo"], r.cfg["tally_Ehi"]
    ie, it = np.meshgrid(np.arange(nE), np.arange(nth), indexing="ij")
    ie, it = ie.ravel(), it.ravel()
    k = lo * (hi / lo) ** ((ie + 0.5) / nE)
    th = (it + 0.5) * math.pi / nth
    w = 1.0 + 0.01 * np.arange(len(k))
    tally(r, k, w, np.cos(th), 0)
    want = np.zeros((nE, nth))
    want[ie, it] = k * w
    assert np.allclose(r.hist_E, want, rtol=1e-14, atol=0)
    want[ie, it] = w
    assert np.allclose(r.hist_N, want, rtol=1e-14, atol=0)
    edge_cases = [
        (lo * (hi / lo) ** (3.0 / nE) * (1 + 1e-12), 1.0, (3, 0)),                # just above an energy edge
        (lo * (hi / lo) ** (7.0 / nE) * (1 - 1e-12), -1.0, (6, nth - 1)),          # just below one; theta = pi
        (lo * 1.000001, math.cos(math.pi * 4.0 / nth + 1e-9), (0, 4)),            # just past an angle edge
    ]
    for kk, dxr, (be, bt) in edge_cases:
        r2 = _tally_run()
        tally(r2, np.array([kk]), np.array([2.0]), np.array([dxr]), 0)
        assert r2.hist_E[be, bt] == pytest.approx(2.0 * kk, rel=1e-14), (kk, dxr, be, bt)
        assert np.count_nonzero(r2.hist_E) == 1
    r3 = _tally_run()
    k3 = np.array([0.5 * lo, hi, 3.0 * hi, 2.0 * W.MEV])
    w3 = np.array([1.0, 2.0, 3.0, 4.0])
    tally(r3, k3, w3, np.ones(4), 2)
    assert r3.flow == pytest.approx([0.5 * lo, 1.0, 2.0 * hi + 9.0 * hi, 5.0], rel=1e-14)
    thr = 2.0 * hi + 9.0 * hi + 8.0 * W.MEV
    assert r3.ledger["photon_thr"] == pytest.approx(thr, rel=1e-14)
    assert r3.series[2] == pytest.approx(thr, rel=1e-14)


def test_gather_reproduces_linear_fields_at_yee_positions():
    check_gather_linear()


def test_gather_wall_ghosts_are_odd_mirrors():
    check_gather_wall_ghosts()


def test_edge_eta_of_linear_resistivity():
    check_edge_eta()


def test_cell_current_sq_of_linear_current():
    check_cell_current_sq()


def test_tally_bins_of_placed_photons():
    check_tally_bins()


def test_deposit_is_the_gathers_adjoint_near_walls():
    """Positions crowded within a half cell of every wall: the deposit is
    the adjoint of the (pinned) gather, so its ghost shares carry the gather's
    indices and signs."""
    rng = np.random.default_rng(21)
    dims = DIMS
    n = 600
    X = rng.uniform(0, 1, size=(n, 3)) * np.array(dims)
    for d in range(3):
        m = rng.uniform(size=n) < 0.5
        X[m, d] = np.where(rng.uniform(size=m.sum()) < 0.5, rng.uniform(0, 0.5, m.sum()),
                           dims[d] - rng.uniform(1e-9, 0.5, m.sum()))
    vel = rng.normal(size=(n, 3)) * 1e8
    w = rng.uniform(0.5, 2, n)
    shape = tuple(d + 1 for d in dims)
    E = tuple(rng.normal(size=shape) for _ in range(3))
    j = tuple(np.zeros(shape) for _ in range(3))
    dx = 1e-6
    PT.deposit(j, X, vel, w, dx, dims)
    Ep, _ = PT.gather(X, E, E, dims)
    lhs = np.sum(PT.Q_E * w[:, None] * vel * Ep)
    rhs = sum(np.sum(j[c] * E[c]) for c in range(3)) * dx ** 3
    assert lhs == pytest.approx(rhs, rel=1e-12)


# ---------------------------------------------------------------------------
# the pins fail on planted mistakes (each a one-character change of a copy)
# ---------------------------------------------------------------------------
def _axis_ghost_sign_plus(X, n, staggered):
    """Copy of the oracle's axis helper with the ghost sign flipped to +1."""
    Xs = X - 0.5 if staggered else X
    i0 = np.floor(Xs).astype(np.int64)
    f = Xs - i0
    i1 = i0 + 1
    s0 = np.ones_like(f)
    s1 = np.ones_like(f)
    if staggered:
        s0 = np.where(i0 < 0, +1.0, 1.0)
        s1 = np.where(i1 > n - 1, -1.0, 1.0)
        i0 = np.clip(i0, 0, n - 1)
        i1 = np.clip(i1, 0, n - 1)
    return i0, i1, f, s0, s1


def _axis_ghost_wrong_index(X, n, staggered):
    """Copy with the upper ghost clamped one index too far in."""
    Xs = X - 0.5 if staggered else X
    i0 = np.floor(Xs).astype(np.int64)
    f = Xs - i0
    i1 = i0 + 1
    s0 = np.ones_like(f)
    s1 = np.ones_like(f)
    if staggered:
        s0 = np.where(i0 < 0, -1.0, 1.0)
        s1 = np.where(i1 > n - 1, -1.0, 1.0)
        i0 = np.clip(i0, 0, n - 1)
        i1 = np.clip(i1, 0, n - 2)
    return i0, i1, f, s0, s1


def _edge_eta_shifted(eta):
    """Copy of edge_eta whose x-edges average cells i+1 instead of i."""
    nx = eta.shape[0]
    ex, ey, ez = F.edge_eta(eta)
    ex = ex.copy()
    ex[:nx - 1] = ex[1:nx]
    return ex, ey, ez


def _ccs_wrong_edge(jh):
    """Copy of cell_current_sq that averages a y-edge pair of jz instead of x."""
    jx, jy, jz = jh
    nx, ny, nz = jx.shape[0] - 1, jx.shape[1] - 1, jx.shape[2] - 1
    cx = 0.25 * (jx[:nx, :ny, :nz] + jx[:nx, 1:, :nz] + jx[:nx, :ny, 1:] + jx[:nx, 1:, 1:])
    cy = 0.25 * (jy[:nx, :ny, :nz] + jy[1:, :ny, :nz] + jy[:nx, :ny, 1:] + jy[1:, :ny, 1:])
    cz = 0.25 * (jz[:nx, :ny, :nz] + jz[:nx, 1:, :nz] + jz[:nx, 1:, :nz] + jz[1:, 1:, :nz])
    return cx * cx + cy * cy + cz * cz


def _tally_angle_from_minus_x(run, k, wph, dirx, n):
    """Copy of the tally with the angle measured from -x."""
    return OracleRun._tally(run, k, wph, -dirx, n)


def _tally_energy_floor_shift(run, k, wph, dirx, n):
    """Copy of the tally whose energy bins start half a bin late."""
    nE = run.hist_E.shape[0]
    lo, hi = run.cfg["tally_Elo"], run.cfg["tally_Ehi"]
    return OracleRun._tally(run, k * (hi / lo) ** (0.5 / nE), wph, dirx, n)


def test_pins_catch_planted_mistakes(monkeypatch):
    cases = []
    # staggering tables: one entry of STAG_B and of STAG_E changed
    bad_b = ((True, True, True),) + PT.STAG_B[1:]
    cases.append(("STAG_B", lambda: monkeypatch.setattr(PT, "STAG_B", bad_b), check_gather_linear))
    bad_e = (PT.STAG_E[0], (False, True, True), PT.STAG_E[2])
    cases.append(("STAG_E", lambda: monkeypatch.setattr(PT, "STAG_E", bad_e), check_gather_linear))
    swap_b = (PT.STAG_B[1], PT.STAG_B[0], PT.STAG_B[2])
    cases.append(("STAG_B swap", lambda: monkeypatch.setattr(PT, "STAG_B", swap_b), check_gather_linear))
    cases.append(("ghost sign", lambda: monkeypatch.setattr(PT, "_axis", _axis_ghost_sign_plus),
                  check_gather_wall_ghosts))
    cases.append(("ghost index", lambda: monkeypatch.setattr(PT, "_axis", _axis_ghost_wrong_index),
                  check_gather_wall_ghosts))
    for name, plant, check in cases:
        plant()
        with pytest.raises(AssertionError):
            check()
        monkeypatch.undo()
    with pytest.raises(AssertionError):
        check_edge_eta(_edge_eta_shifted)
    with pytest.raises(AssertionError):
        check_cell_current_sq(_ccs_wrong_edge)
    with pytest.raises(AssertionError):
        check_tally_bins(_tally_angle_from_minus_x)
    with pytest.raises(AssertionError):
        check_tally_bins(_tally_energy_floor_shift)
    # and the unmutated pieces pass
    check_gather_linear()
    check_gather_wall_ghosts()
