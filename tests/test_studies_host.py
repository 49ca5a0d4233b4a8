"""Host-side logic of the physics studies: the viscosity-rate relation the
paper prints, and the contact-angle and Laplace-fit measurements on
synthetic fields with known answers."""
import math

import numpy as np
import pytest

from paper_1805_08643_amd import studies


@pytest.mark.parametrize("nu,inv_s", [(0.01, 0.53), (0.1, 0.8), (0.15, 0.95)])
def test_tau_for_nu_matches_printed_pairs(nu, inv_s):
    # Sec. IV.B and IV.D pair nu = 0.1 with 1/s_nu = 0.8 and the range
    # 0.01..0.15 with 0.53..0.95.
    assert studies.tau_for_nu(nu) == pytest.approx(inv_s, abs=1e-12)


@pytest.mark.parametrize("zc,R", [(5.0, 20.0), (-8.0, 24.0), (14.0, 18.0)])
def test_contact_angle_of_synthetic_cap(zc, R):
    nx = ny = 80
    nz = 50
    x = np.arange(nx)[None, None, :] - 40.0
    y = np.arange(ny)[None, :, None] - 40.5
    z = np.arange(nz)[:, None, None] - zc
    r = np.sqrt(x * x + y * y + z * z)
    rl, rv = 2.0, 0.3
    rho = 0.5 * (rl + rv) - 0.5 * (rl - rv) * np.tanh(2.0 * (r - R) / 4.0)
    for zw in (0.0, -0.5):
        want = math.degrees(math.acos((zw - zc) / R))
        got, fit = studies.contact_angle(rho.reshape(-1), nx, ny, nz, 0.5 * (rl + rv), zw=zw)
        assert got == pytest.approx(want, abs=0.5)
        assert fit["cap_formula_deg"] == pytest.approx(want, abs=0.5)
        assert fit["radius"] == pytest.approx(R, abs=0.3)


def test_linfit_recovers_line():
    x = np.array([0.02, 0.03, 0.05, 0.07])
    s, b, r2 = studies._linfit(x, 0.3 * x - 1e-4)
    assert s == pytest.approx(0.3) and b == pytest.approx(-1e-4, abs=1e-12) and r2 == pytest.approx(1.0)


def test_bulk_plateaus():
    rho = np.concatenate([np.full(100, 2.8), np.linspace(0.4, 2.8, 50), np.full(100, 0.37)])
    rl, rv = studies._bulk(rho)
    assert rl == pytest.approx(2.8, abs=1e-3) and rv == pytest.approx(0.37, abs=1e-3)
