"""Hybrid field solver on a Yee grid (App. A of the paper):
  E = eta (curl B / mu0 - j_h)        eq. (Ampere_Maxwell) with eq. (Ohms_Law)
  dB/dt = -curl E                     eq. (Faraday_Lens)
Oracle-only implementation, FP64, SI.

Grid: nx*ny*nz cubic cells of side dx; nodes (i, j, k), i in [0, nx].
Every component lives in an array of shape (nx+1, ny+1, nz+1):
  Ex[i,j,k] at (i+1/2, j, k)      Bx[i,j,k] at (i, j+1/2, k+1/2)
  Ey[i,j,k] at (i, j+1/2, k)      By[i,j,k] at (i+1/2, j, k+1/2)
  Ez[i,j,k] at (i, j, k+1/2)      Bz[i,j,k] at (i+1/2, j+1/2, k)
j_h shares the E positions.  Entries past a staggered range stay zero.
Cell-centred eta has shape (nx, ny, nz); eta = 0 outside the solid.

Boundaries (reading; the paper does not state them).  The reflux walls
mirror the electrons, so the fields take the mirror symmetry of a wall: a
component that is staggered along an axis (E or j normal to the wall, B
tangential to it) is odd about the wall, i.e. its value one half-cell
outside the grid is minus the nearest value inside.  This sets B_t = 0 on
the walls, so no Poynting flux crosses them.  The cell-centred eta is even:
edges on a wall average the clamped (nearest) cells.
"""
from __future__ import annotations

import numpy as np

from . import constants as K


def _cl(idx, n):
    return np.clip(idx, 0, n - 1)


def edge_eta(eta):
    """Resistivity on the three edge families: the mean of the four cells that
    share the edge (clamped at the domain faces).  Returns (ex, ey, ez) each
    of shape (nx+1, ny+1, nz+1)."""
    nx, ny, nz = eta.shape
    out = []
    I = np.arange(nx + 1)[:, None, None]
    J = np.arange(ny + 1)[None, :, None]
    Kk = np.arange(nz + 1)[None, None, :]
    # x-edges (i+1/2, j, k): cells (i, j-1|j, k-1|k)
    i = np.minimum(I, nx - 1)
    ex = 0.25 * (eta[i, _cl(J - 1, ny), _cl(Kk - 1, nz)] + eta[i, _cl(J, ny), _cl(Kk - 1, nz)]
                 + eta[i, _cl(J - 1, ny), _cl(Kk, nz)] + eta[i, _cl(J, ny), _cl(Kk, nz)])
    ex = np.where(I < nx, ex, 0.0)
    j = np.minimum(J, ny - 1)
    ey = 0.25 * (eta[_cl(I - 1, nx), j, _cl(Kk - 1, nz)] + eta[_cl(I, nx), j, _cl(Kk - 1, nz)]
                 + eta[_cl(I - 1, nx), j, _cl(Kk, nz)] + eta[_cl(I, nx), j, _cl(Kk, nz)])
    ey = np.where(J < ny, ey, 0.0)
    k = np.minimum(Kk, nz - 1)
    ez = 0.25 * (eta[_cl(I - 1, nx), _cl(J - 1, ny), k] + eta[_cl(I, nx), _cl(J - 1, ny), k]
                 + eta[_cl(I - 1, nx), _cl(J, ny), k] + eta[_cl(I, nx), _cl(J, ny), k])
    ez = np.where(Kk < nz, ez, 0.0)
    out = (ex, ey, ez)
    return out


def curl_B(B, dx):
    """curl B on the E positions (odd ghosts for B tangential to a wall)."""
    Bx, By, Bz = B
    n1 = Bx.shape
    nx, ny, nz = n1[0] - 1, n1[1] - 1, n1[2] - 1
    I = np.arange(nx + 1)[:, None, None]
    J = np.arange(ny + 1)[None, :, None]
    Kk = np.arange(nz + 1)[None, None, :]

    def sg(idx, n):
        return np.where((idx < 0) | (idx > n - 1), -1.0, 1.0)

    # x: (dBz/dy - dBy/dz) at (i+1/2, j, k); Bz staggered in y, By staggered in z
    i = np.minimum(I, nx - 1)
    cx = ((sg(J, ny) * Bz[i, _cl(J, ny), Kk] - sg(J - 1, ny) * Bz[i, _cl(J - 1, ny), Kk])
          - (sg(Kk, nz) * By[i, J, _cl(Kk, nz)] - sg(Kk - 1, nz) * By[i, J, _cl(Kk - 1, nz)])) / dx
    cx = np.where(I < nx, cx, 0.0)
    # y: (dBx/dz - dBz/dx) at (i, j+1/2, k); Bx staggered in z, Bz staggered in x
    j = np.minimum(J, ny - 1)
    cy = ((sg(Kk, nz) * Bx[I, j, _cl(Kk, nz)] - sg(Kk - 1, nz) * Bx[I, j, _cl(Kk - 1, nz)])
          - (sg(I, nx) * Bz[_cl(I, nx), j, Kk] - sg(I - 1, nx) * Bz[_cl(I - 1, nx), j, Kk])) / dx
    cy = np.where(J < ny, cy, 0.0)
    # z: (dBy/dx - dBx/dy) at (i, j, k+1/2); By staggered in x, Bx staggered in y
    k = np.minimum(Kk, nz - 1)
    cz = ((sg(I, nx) * By[_cl(I, nx), J, k] - sg(I - 1, nx) * By[_cl(I - 1, nx), J, k])
          - (sg(J, ny) * Bx[I, _cl(J, ny), k] - sg(J - 1, ny) * Bx[I, _cl(J - 1, ny), k])) / dx
    cz = np.where(Kk < nz, cz, 0.0)
    return cx, cy, cz


def curl_E(E, dx):
    """curl E on the B positions; every face is surrounded by grid edges."""
    Ex, Ey, Ez = E
    n1 = Ex.shape
    nx, ny, nz = n1[0] - 1, n1[1] - 1, n1[2] - 1
    cx = np.zeros(n1)
    cy = np.zeros(n1)
    cz = np.zeros(n1)
    # Bx at (i, j+1/2, k+1/2): dEz/dy - dEy/dz
    cx[:, :ny, :nz] = ((Ez[:, 1:ny + 1, :nz] - Ez[:, :ny, :nz])
                       - (Ey[:, :ny, 1:nz + 1] - Ey[:, :ny, :nz])) / dx
    # By at (i+1/2, j, k+1/2): dEx/dz - dEz/dx
    cy[:nx, :, :nz] = ((Ex[:nx, :, 1:nz + 1] - Ex[:nx, :, :nz])
                       - (Ez[1:nx + 1, :, :nz] - Ez[:nx, :, :nz])) / dx
    # Bz at (i+1/2, j+1/2, k): dEy/dx - dEx/dy
    cz[:nx, :ny, :] = ((Ey[1:nx + 1, :ny, :] - Ey[:nx, :ny, :])
                       - (Ex[:nx, 1:ny + 1, :] - Ex[:nx, :ny, :])) / dx
    return cx, cy, cz


def ohm(B, jh, eta, dx):
    """E = eta_edge (curl B / mu0 - j_h)."""
    ee = edge_eta(eta)
    cb = curl_B(B, dx)
    return tuple(ee[c] * (cb[c] / K.MU0 - jh[c]) for c in range(3))


def faraday(B, E, dt, dx):
    """B <- B - dt curl E."""
    ce = curl_E(E, dx)
    return tuple(B[c] - dt * ce[c] for c in range(3))


def field_update(E, B, jh, eta, dt, dx, n_sub, evolve_e=True, evolve_b=True):
    """n_sub sub-cycles of (Ohm, Faraday) with dt/n_sub each."""
    for _ in range(n_sub):
        if evolve_e:
            E = ohm(B, jh, eta, dx)
        if evolve_b:
            B = faraday(B, E, dt / n_sub, dx)
    return E, B


def div_B(B, dx):
    """Divergence of B at cell centres (i+1/2, j+1/2, k+1/2)."""
    Bx, By, Bz = B
    nx, ny, nz = Bx.shape[0] - 1, Bx.shape[1] - 1, Bx.shape[2] - 1
    return ((Bx[1:nx + 1, :ny, :nz] - Bx[:nx, :ny, :nz])
            + (By[:nx, 1:ny + 1, :nz] - By[:nx, :ny, :nz])
            + (Bz[:nx, :ny, 1:nz + 1] - Bz[:nx, :ny, :nz])) / dx


def cell_current_sq(jh):
    """|j_h|^2 at cell centres: each component is the mean of the four edges of
    the cell parallel to it."""
    jx, jy, jz = jh
    nx, ny, nz = jx.shape[0] - 1, jx.shape[1] - 1, jx.shape[2] - 1
    cx = 0.25 * (jx[:nx, :ny, :nz] + jx[:nx, 1:, :nz] + jx[:nx, :ny, 1:] + jx[:nx, 1:, 1:])
    cy = 0.25 * (jy[:nx, :ny, :nz] + jy[1:, :ny, :nz] + jy[:nx, :ny, 1:] + jy[1:, :ny, 1:])
    cz = 0.25 * (jz[:nx, :ny, :nz] + jz[1:, :ny, :nz] + jz[:nx, 1:, :nz] + jz[1:, 1:, :nz])
    return cx * cx + cy * cy + cz * cz
