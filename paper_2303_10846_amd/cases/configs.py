"""Synthetic workloads standing in for the paper's cases (Sec. 4).

Every quantity is dimensionless in the system of Sec. 4 (L_ref = L_c,
rho_ref = rho_inf, T_ref = T_inf, U_ref = sqrt(2 R T_ref)), so the gas constant
is R = 1/2 and the free stream has rho = T = 1.

A case is a plain dict: mesh arrays, the DVS, the gas and numerics constants,
the boundary conditions and the initial macroscopic state.  The solver
library and the CPU oracle read the same dict.
"""
from __future__ import annotations

import math

import numpy as np

from . import dvs as _dvs
from . import mesh as _mesh

__all__ = ["gas_n2", "numerics_default", "mu_ref_from_kn", "cavity_case", "sphere_case", "sphere_hex_case",
           "small_sphere_hex_case",
           "capsule_case", "capsule_hex_case",
           "freestream_box_case", "open_box_case", "small_sphere_case", "rest_state"]

WALL = 1
FARFIELD = 2


def mu_ref_from_kn(kn: float, omega: float) -> float:
    """Reference viscosity from the Knudsen number for VHS molecules.

    Dimensionless form of the VHS mean free path (Bird), lambda =
    2(5-2w)(7-2w)/15 * mu / (rho sqrt(2 pi R T)), with rho = T = 1, R = 1/2,
    lambda = Kn.
    """
    return 15.0 * math.sqrt(math.pi) * kn / (2.0 * (5.0 - 2.0 * omega) * (7.0 - 2.0 * omega))


def gas_n2(kn: float, z_rot: float = 3.0, omega: float = 0.74):
    """Nitrogen, Rykov model; delta, omega0, omega1 are the N2 constants of the Rykov-model literature."""
    return dict(R=0.5, gamma=1.4, Z=z_rot, delta=1.0 / 1.55, omega0=0.2354, omega1=0.3049,
                mu_ref=mu_ref_from_kn(kn, omega), omega_vhs=omega, T_ref=1.0, Kn=kn)


def numerics_default():
    return dict(cfl=0.5, inv_dt=0.0, cfl_imp=0.0, lim_K=1.0, limiter=1, n_macro=40, n_micro=2,
                snap=1e-13, macro_exact_jvp=0)


def rest_state(rho=1.0, U=(0.0, 0.0, 0.0), T=1.0, R=0.5):
    """W = (rho, rho U, rho E, rho E_rot) of an equilibrium gas (T_tr = T_rot = T)."""
    U = np.asarray(U, dtype=float)
    rE = 0.5 * rho * float(U @ U) + 2.5 * rho * R * T
    return np.array([rho, rho * U[0], rho * U[1], rho * U[2], rE, rho * R * T])


def _bc(tag, kind, rho=1.0, U=(0.0, 0.0, 0.0), T=1.0):
    return dict(tag=int(tag), kind=int(kind), rho=float(rho), U=[float(x) for x in U], T=float(T))


def _box(kind, n, seed, tag_of_plane=None):
    """Box mesh of n^3 grid cells: "tet" (6 Kuhn tetrahedra each), "hex" (the hexahedra themselves) or "mixed"
    (hexahedra, pyramids and tetrahedra)."""
    if kind == "tet":
        return _mesh.kuhn_box_mesh(n=n, seed=seed, tag_of_plane=tag_of_plane)
    if kind == "hex":
        return _mesh.hex_box_mesh(n=n, seed=seed, tag_of_plane=tag_of_plane)
    if kind == "mixed":
        return _mesh.mixed_box_mesh(n=n, seed=seed, tag_of_plane=tag_of_plane)
    raise ValueError(f"unknown mesh kind {kind}")


def cavity_case(seed: int = 0, n: int = 6, nv_side: int = 8, kn: float = 0.1, lid_speed: float = 0.15,
                n_iter: int = 200, kind: str = "tet"):
    """3-D lid-driven cubic cavity: n^3 hexes x 6 Kuhn tets (kind "hex": the hexes, "mixed": hexes, pyramids and
    tets), Cartesian nv_side^3 DVS on [-4,4]^3."""
    m = _box(kind, n, seed)
    u, w = _dvs.cartesian_dvs(nv_side, 4.0)
    gas = gas_n2(kn, 3.0)
    bcs = [_bc(1, WALL, U=(0, 0, 0), T=1.0), _bc(2, WALL, U=(lid_speed, 0, 0), T=1.0)]
    W0 = rest_state()
    return dict(name=f"cavity{n}^3_{kind}_dvs{nv_side}^3_kn{kn}_seed{seed}", mesh=m, u=u, w=w, gas=gas,
                num=numerics_default(), bcs=bcs, W0=W0, n_iter=n_iter)


def freestream_box_case(seed: int = 0, n: int = 3, U=(0.3, -0.1, 0.2), dvs=None, kn: float = 0.1,
                        kind: str = "tet"):
    """All-far-field box: a uniform free stream must give a zero residual."""
    m = _box(kind, n, seed, tag_of_plane=lambda a, s: 2)
    if dvs is None:
        u, w = _dvs.cartesian_dvs(8, 4.0)
    else:
        u, w = dvs
    gas = gas_n2(kn, 3.0)
    bcs = [_bc(2, FARFIELD, rho=1.0, U=U, T=1.0)]
    return dict(name=f"freestream_box{n}_{kind}", mesh=m, u=u, w=w, gas=gas, num=numerics_default(), bcs=bcs,
                W0=rest_state(1.0, U, 1.0), n_iter=1)


def open_box_case(seed: int = 0, n: int = 3, U=(0.3, 0.0, 0.0), T_wall: float = 1.5, nv_side: int = 6,
                  kn: float = 0.1, kind: str = "tet"):
    """Box with a diffuse wall at z = 0 (tag 1) and far field on the other five sides (tag 2).

    Unlike the closed cavity, whose steady states form a family parameterised by
    the total mass, this problem has a unique steady state.
    """
    m = _box(kind, n, seed, tag_of_plane=lambda a, s: 1 if (a == 2 and s == 0) else 2)
    u, w = _dvs.cartesian_dvs(nv_side, 4.0)
    gas = gas_n2(kn, 3.0)
    bcs = [_bc(1, WALL, U=(0, 0, 0), T=T_wall), _bc(2, FARFIELD, rho=1.0, U=U, T=1.0)]
    return dict(name=f"open_box{n}_{kind}", mesh=m, u=u, w=w, gas=gas, num=numerics_default(), bcs=bcs,
                W0=rest_state(1.0, U, 1.0), n_iter=100)


def _external_case(name, body, n_ang, n_rad, r_far, first_layer, mach, kn, z_rot, tw, nv_target,
                   seed, n_iter, h_outer=None, refine_scale=1.0, smooth_passes=0, jitter=0.1, cells="tet"):
    gamma = 1.4
    R = 0.5
    uinf = mach * math.sqrt(gamma * R * 1.0)
    U = np.array([uinf, 0.0, 0.0])
    m = _mesh.shell_mesh(body, n_ang=n_ang, n_rad=n_rad, r_far=r_far, first_layer=first_layer, seed=seed,
                         smooth_passes=smooth_passes, jitter=jitter, cells=cells)
    u, w = _dvs.paper_unstructured_dvs(U, 1.0, tw, mach, 5.0, h_outer=h_outer, target=nv_target,
                                       refine_scale=refine_scale)
    gas = gas_n2(kn, z_rot)
    bcs = [_bc(1, WALL, U=(0, 0, 0), T=tw), _bc(2, FARFIELD, rho=1.0, U=U, T=1.0)]
    # Start from gas at rest at the free-stream density and temperature; the free stream enters
    # through the far field.  A finite implicit step (CFL_imp = 5) keeps the first hypersonic
    # iterations from emptying the wake cells.
    num = dict(numerics_default(), cfl_imp=5.0)
    return dict(name=name, mesh=m, u=u, w=w, gas=gas, num=num, bcs=bcs,
                W0=rest_state(1.0, (0.0, 0.0, 0.0), 1.0), n_iter=n_iter, mach=mach, U_inf=U, T_w=tw)


def sphere_case(seed: int = 0, n_ang: int = 10, n_rad: int = 7, nv_target: int = 4096, n_iter: int = 200):
    """Ma 5 flow over a unit-diameter sphere at Kn = 0.1, Tw/T_inf = 3 (~50k tets x ~4k velocities)."""
    return _external_case(f"sphere_ma5_kn0.1_{n_ang}x{n_rad}_seed{seed}", _mesh.sphere_body(0.5), n_ang, n_rad,
                          3.0, 0.03, 5.0, 0.1, 3.0, 3.0, nv_target, seed, n_iter)


def sphere_hex_case(seed: int = 0, n_ang: int = 24, n_rad: int = 14, nv_target: int = 4096, n_iter: int = 200):
    """The sphere case on the hexahedral O-grid itself (the paper's sphere mesh is hexahedral, Sec. 4.2):
    6 x 24 x 24 x 14 = 48 384 hexahedra graded from 0.03 at the wall, the same DVS and flow."""
    return _external_case(f"sphere_hex_ma5_kn0.1_{n_ang}x{n_rad}_seed{seed}", _mesh.sphere_body(0.5), n_ang, n_rad,
                          3.0, 0.03, 5.0, 0.1, 3.0, 3.0, nv_target, seed, n_iter, cells="hex")


def small_sphere_case(seed: int = 0, n_ang: int = 3, n_rad: int = 3, h_outer: float = 2.2, refine_scale: float = 2.0,
                      n_iter: int = 20):
    """About 2k tets and a few hundred velocities with the sphere's physics (parity-test size)."""
    return _external_case(f"sphere_small_{n_ang}x{n_rad}_seed{seed}", _mesh.sphere_body(0.5), n_ang, n_rad,
                          3.0, 0.1, 5.0, 0.1, 3.0, 3.0, None, seed, n_iter, h_outer=h_outer,
                          refine_scale=refine_scale)


def small_sphere_hex_case(seed: int = 0, n_ang: int = 4, n_rad: int = 4, h_outer: float = 2.2,
                          refine_scale: float = 2.0, n_iter: int = 20):
    """A few hundred hexahedra with the small sphere's DVS and physics (parity-test size)."""
    return _external_case(f"sphere_hex_small_{n_ang}x{n_rad}_seed{seed}", _mesh.sphere_body(0.5), n_ang, n_rad,
                          3.0, 0.1, 5.0, 0.1, 3.0, 3.0, None, seed, n_iter, h_outer=h_outer,
                          refine_scale=refine_scale, cells="hex")


def capsule_case(seed: int = 0, n_ang: int = 18, n_rad: int = 13, nv_target: int = 10000, n_iter: int = 50,
                 smooth_passes: int = 4):
    """Ma 10 blunt capsule (spherical-cap forebody, 33 deg aftbody) at Kn = 0.01 (~300k tets x ~10k velocities).

    Z_rot and Tw/T_inf borrow the paper's Ma 10.15 N2 blunted-cone conditions
    (Z_rot = 4.24, Tw/T_inf = 600/143.5).
    """
    # the wall radius is smoothed over the ray grid: a rounded shoulder instead of a sharp cap/cone edge
    c = _external_case(f"capsule_ma10_kn0.01_{n_ang}x{n_rad}_seed{seed}", _mesh.capsule_body(), n_ang, n_rad,
                       3.0, 0.01, 10.0, 0.01, 4.24, 600.0 / 143.5, nv_target, seed, n_iter,
                       smooth_passes=smooth_passes, jitter=0.03)
    c["num"]["cfl_imp"] = 1.0  # Ma 10 from rest: a smaller implicit step keeps the first predictions positive
    return c


def capsule_hex_case(seed: int = 0, n_ang: int = 18, n_rad: int = 13, nv_target: int = 10000, n_iter: int = 50,
                     smooth_passes: int = 4):
    """The Ma 10 capsule on the hexahedral O-grid that the tetrahedral capsule splits into 12 tets per cell
    (6 x 18 x 18 x 13 = 25 272 hexahedra), with the same body, jitter, DVS, gas and boundaries.  The paper's
    blunted-cone mesh is hexahedral (Sec. 4.3)."""
    c = _external_case(f"capsule_hex_ma10_kn0.01_{n_ang}x{n_rad}_seed{seed}", _mesh.capsule_body(), n_ang, n_rad,
                       3.0, 0.01, 10.0, 0.01, 4.24, 600.0 / 143.5, nv_target, seed, n_iter,
                       smooth_passes=smooth_passes, jitter=0.03, cells="hex")
    c["num"]["cfl_imp"] = 1.0
    return c
