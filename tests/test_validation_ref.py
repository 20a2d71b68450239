"""The rotational validation's reference values (CPU): the Tirado formula
(Eqs. CapsTheorRotatMotionTirado and EndeffCorrRotatMotionTirado) and the
unit conversion of the validation driver against the values the paper
prints (tests/golden/rotation_validation.json, cited there)."""
import json
import os

import numpy as np

from paper_1503_06869_amd import validation as V

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rotation_validation.json")))


def test_parameters_are_the_papers():
    assert V.DX == GOLD["dx_m"] and V.NU == GOLD["nu_m2_s"] and V.TAU == GOLD["tau"]
    assert V.RHO_F == GOLD["rho_f_kg_m3"] and V.RHO_P == GOLD["rho_p_kg_m3"]
    assert V.R_CELLS == GOLD["radius_dx"]
    # dt = 183e-6 s as the paper states (Eq. kinVisc with tau = 6)
    assert abs(V.dt() - 183e-6) < 0.5e-6
    for A, L in zip(GOLD["aspect_ratios"], GOLD["length_m"]):
        assert abs(A * V.R_CELLS * V.DX - L) < 1e-12


def test_tirado_rotation_reproduces_the_printed_values():
    """omega = M / gamma_r for cylinders of the full length (wC) and of the
    length without the caps L - 2r (nC), to the printed three digits."""
    r = V.R_CELLS * V.DX
    for i, A in enumerate(GOLD["aspect_ratios"]):
        M = GOLD["torque_1e-15_kg_m2_s2"][i] * 1e-15
        L = GOLD["length_m"][i]
        wc = V.tirado_rotation(M, L, r)
        nc = V.tirado_rotation(M, L - 2 * r, r)
        assert abs(wc / GOLD["omega_tirado_wc_per_s"][i] - 1) < 5e-3, (A, wc)
        assert abs(nc / GOLD["omega_tirado_nc_per_s"][i] - 1) < 5e-3, (A, nc)


def test_lattice_units_round_trip():
    """Torque and angular velocity in lattice units: M_lat = M dt^2 /
    (rho_f dx^5); an angular velocity omega [1/s] is omega dt per step."""
    M = 12.26e-15
    m_lat = V.lattice_torque(M)
    np.testing.assert_allclose(m_lat * V.RHO_F * V.DX ** 5 / V.dt() ** 2, M, rtol=1e-14)
