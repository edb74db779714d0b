"""Wall coefficients (Eqs. 70-72 and the force and moment coefficients) from per-face loads: the library's host
arithmetic (cis_wall_coefficients_of_loads), which needs no GPU.

Synthetic loads on the six unit faces of a cube of side 1 centred at the origin, with n pointing from the gas
into the body: a uniform pressure gives no net force and no moment; a shear tau0 e_z on the face x = +1/2 gives
the force tau0 e_z and the moment (e_x / 2) x (tau0 e_z) = -tau0 / 2 e_y about the centre.
"""
import numpy as np

from paper_2303_10846_amd.binding import wall_coefficients


def _cube_loads(p0, tau0):
    x, n = [], []
    for ax in range(3):
        for sg in (1.0, -1.0):
            e = np.zeros(3)
            e[ax] = sg
            x.append(0.5 * e)
            n.append(-e)
    x, n = np.array(x), np.array(n)
    area = np.ones(6)
    p = np.full(6, p0)
    tau = np.zeros((6, 3))
    tau[0] = [0.0, 0.0, tau0]          # face x = +1/2, n = -e_x
    f = area[:, None] * (p[:, None] * n + tau)
    return dict(x=x, area=area, n=n, p=p, tau=tau, q=np.full(6, 0.25), force=f.sum(axis=0), heat=1.5)


def test_uniform_pressure_gives_no_force_and_no_moment():
    L = _cube_loads(p0=2.0, tau0=0.0)
    rho, U, T, R = 1.0, (3.0, 0.0, 0.0), 1.0, 0.5
    c = wall_coefficients(L, rho, U, T, R=R, A_ref=1.0)
    qd = 0.5 * rho * 9.0
    assert np.allclose(c["Cp"], (2.0 - rho * R * T) / qd, rtol=0, atol=1e-15)
    assert np.allclose(c["Ctau"], 0.0) and np.allclose(c["Ch"], 0.25 / (qd * 3.0))
    assert abs(c["Cd"]) < 1e-15 and abs(c["Cl"]) < 1e-15
    assert np.max(np.abs(c["CM"])) < 1e-15 and abs(c["Cm"]) < 1e-15
    assert abs(c["CQ"] - 1.5 / (qd * 3.0)) < 1e-15


def test_shear_gives_lift_and_pitching_moment():
    tau0 = 0.3
    L = _cube_loads(p0=1.0, tau0=tau0)
    rho, U, T = 1.0, (2.0, 0.0, 0.0), 1.0
    qd = 0.5 * rho * 4.0
    c = wall_coefficients(L, rho, U, T, A_ref=2.0, L_ref=0.5)
    assert abs(c["Cd"]) < 1e-15
    assert abs(c["Cl"] - tau0 / (qd * 2.0)) < 1e-15                     # e_L = z
    assert np.allclose(c["CM"], [0.0, -0.5 * tau0 / (qd * 2.0 * 0.5), 0.0], rtol=0, atol=1e-15)
    assert abs(c["Cm"] - c["CM"][1]) < 1e-15                            # e_L x e_D = z x x = y
    assert np.allclose(c["Ctau"][0], tau0 / qd) and np.allclose(c["Ctau"][1:], 0.0)
    # moment about another point: M(x1) = M(x0) + (x0 - x1) x F
    x1 = np.array([0.2, -0.1, 0.4])
    c1 = wall_coefficients(L, rho, U, T, A_ref=2.0, L_ref=0.5, x_ref=x1)
    F = L["force"]
    assert np.allclose(c1["CM"] * qd * 2.0 * 0.5, c["CM"] * qd * 2.0 * 0.5 + np.cross(-x1, F), rtol=0, atol=1e-14)


def test_lift_direction_defaults_to_y_when_the_flow_is_along_z():
    L = _cube_loads(p0=1.0, tau0=0.0)
    L["tau"][0] = [0.0, 0.7, 0.0]                                       # a shear along y on the face x = +1/2
    c = wall_coefficients(L, 1.0, (0.0, 0.0, 2.0), 1.0, A_ref=1.0)
    assert np.allclose(c["force"], [0.0, 0.7, 0.0], rtol=0, atol=1e-15)
    assert abs(c["Cl"] - 0.7 / 2.0) < 1e-15 and abs(c["Cd"]) < 1e-15
    assert np.allclose(c["e_lift"], [0.0, 1.0, 0.0]) and np.allclose(c["e_drag"], [0.0, 0.0, 1.0])


def test_bad_references_are_rejected():
    import pytest
    from paper_2303_10846_amd.binding import CisError
    L = _cube_loads(p0=1.0, tau0=0.0)
    for kw in (dict(rho_inf=0.0), dict(U_inf=(0.0, 0.0, 0.0)), dict(T_inf=-1.0)):
        args = dict(rho_inf=1.0, U_inf=(1.0, 0.0, 0.0), T_inf=1.0)
        args.update(kw)
        with pytest.raises(CisError) as e:
            wall_coefficients(L, args["rho_inf"], args["U_inf"], args["T_inf"], A_ref=1.0)
        assert e.value.status == -1
    with pytest.raises(CisError):
        wall_coefficients(L, 1.0, (1.0, 0.0, 0.0), 1.0, A_ref=1.0, lift_dir=(2.0, 0.0, 0.0))
