"""Contact angle of a sessile drop from a density field (TEST INFRASTRUCTURE ONLY).

Sec. V: with base width L and height H of the spherical cap, the radius is
R = (4 H^2 + L^2) / (8 H) and tan(theta) = L / (2 (R - H)).

Readings (the paper gives only the formula): the interface is the rho_mid
isoline; L is the liquid width on the base row, with both edges located by
linear interpolation between the last liquid and the first vapour node; H is
measured on the drop's symmetry column (the column nearest the centre of the
excess mass), from the surface height to the interpolated top crossing;
theta = atan2(L/2, R - H) so that angles above 90 degrees (R < H) come out
right.  A drop that does not wet the base row has L = 0 and theta = 180.
"""
from __future__ import annotations

import math

import numpy as np


def _crossing(x_liq, r_liq, x_vap, r_vap, mid):
    """Linear interpolation of the point where rho = mid between two nodes."""
    return x_liq + (mid - r_liq) / (r_vap - r_liq) * (x_vap - x_liq)


def contact_angle(rho, rho_mid, base_row=1, surface_y=None):
    """(theta_deg, L, H, R) of the drop sitting on ``base_row`` of rho[ny][nx].

    ``surface_y`` is the height that H is measured from (default: base_row)."""
    rho = np.asarray(rho, dtype=np.float64)
    ny, nx = rho.shape
    if surface_y is None:
        surface_y = float(base_row)
    liquid = rho > rho_mid
    excess = np.where(liquid, rho - rho_mid, 0.0)
    excess[:base_row, :] = 0.0
    tot = excess.sum()
    if tot <= 0.0:
        return float("nan"), 0.0, 0.0, 0.0
    xc = float((excess.sum(axis=0) * np.arange(nx)).sum() / tot)
    ic = int(round(xc)) % nx

    # height on the symmetry column: walk up from the base row through liquid
    col = rho[:, ic]
    y = base_row
    while y < ny and not col[y] > rho_mid:
        y += 1
    y_bottom_liq = y
    while y + 1 < ny and col[y + 1] > rho_mid:
        y += 1
    if y_bottom_liq >= ny:
        return float("nan"), 0.0, 0.0, 0.0
    y_top = _crossing(y, col[y], y + 1, col[y + 1], rho_mid) if y + 1 < ny else float(y)
    H = y_top - surface_y

    # base width on the base row
    row = rho[base_row, :]
    if not row[ic] > rho_mid:
        return 180.0, 0.0, H, H / 2.0
    xl = ic
    while row[(xl - 1) % nx] > rho_mid and ic - xl < nx:
        xl -= 1
    xr = ic
    while row[(xr + 1) % nx] > rho_mid and xr - ic < nx:
        xr += 1
    x_left = _crossing(xl, row[xl % nx], xl - 1, row[(xl - 1) % nx], rho_mid)
    x_right = _crossing(xr, row[xr % nx], xr + 1, row[(xr + 1) % nx], rho_mid)
    L = x_right - x_left

    R = (4.0 * H * H + L * L) / (8.0 * H)
    theta = math.degrees(math.atan2(L / 2.0, R - H))
    return theta, L, H, R
