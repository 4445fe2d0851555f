"""Pins of the oracle's contact-angle measurement (Sec. V formula) on synthetic
spherical caps of known angle, and of the geometry identities it uses."""
import math

import numpy as np
import pytest

from oracle.contact import contact_angle


def cap_field(nx, ny, Rc, theta_deg, surface_y=1.0, rho_l=7.0, rho_g=0.2, width=3.0):
    """Circular cap of radius Rc cut by the plane y = surface_y at angle theta: the
    circle's centre sits at surface_y - Rc cos(theta)."""
    th = math.radians(theta_deg)
    cx, cy = nx / 2.0, surface_y - Rc * math.cos(th)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    r = np.hypot(x - cx, y - cy)
    return 0.5 * (rho_l + rho_g) - 0.5 * (rho_l - rho_g) * np.tanh(2 * (r - Rc) / width)


@pytest.mark.parametrize("theta", [30, 45, 60, 90, 105, 120, 135, 150])
def test_synthetic_caps(theta):
    rho = cap_field(400, 220, 60.0, theta)
    th, L, H, R = contact_angle(rho, 0.5 * (7.0 + 0.2), base_row=1)
    assert abs(th - theta) < 0.5
    assert abs(R - 60.0) < 1.0


def test_geometry_identities():
    """R = (4H^2 + L^2)/(8H) is the circle through the base ends and the apex."""
    for Rc, theta in ((50.0, 40.0), (30.0, 120.0)):
        th = math.radians(theta)
        L = 2 * Rc * math.sin(th)
        H = Rc * (1 - math.cos(th))
        assert abs((4 * H * H + L * L) / (8 * H) - Rc) < 1e-12
        assert abs(math.degrees(math.atan2(L / 2, Rc - H)) - theta) < 1e-10


def test_detached_drop_is_180():
    rho = cap_field(200, 150, 30.0, 180.0, surface_y=8.0)  # lowest point at y = 8
    th, L, H, R = contact_angle(rho, 3.6, base_row=1)
    assert th == 180.0 and L == 0.0
