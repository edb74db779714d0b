"""Discrete velocity sets (points u_k, weights w_k) for the synthetic workloads.

A discrete velocity is the centroid of a cell of the velocity-space mesh and
its weight is that cell's volume (Sec. 3.2, text after Eq. 37).  This module
only builds those arrays; it holds none of the scheme's arithmetic.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["cartesian_dvs", "octree_dvs", "gauss_hermite_dvs", "total_temperature",
           "refine_weight", "refine_count", "paper_unstructured_dvs"]


def cartesian_dvs(n: int = 8, half_width: float = 4.0):
    """Midpoints of an n^3 uniform grid on [-L, L]^3; weights are the cell volumes."""
    h = 2.0 * half_width / n
    c = -half_width + h * (np.arange(n) + 0.5)
    U, V, W = np.meshgrid(c, c, c, indexing="ij")
    u = np.stack([U.ravel(), V.ravel(), W.ravel()], axis=1)
    w = np.full(len(u), h ** 3)
    return u, w


def gauss_hermite_dvs(n: int, U, T: float, R: float = 0.5):
    """Tensor Gauss-Hermite set scaled to a Maxwellian of temperature T at mean U.

    Integrates (Maxwellian at T, U) x (polynomial of degree <= 2n-1 per axis)
    exactly up to rounding.
    """
    x, wx = np.polynomial.hermite_e.hermegauss(n)
    sig = math.sqrt(R * T)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    WX, WY, WZ = np.meshgrid(wx, wx, wx, indexing="ij")
    xx = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    w = (WX * WY * WZ).ravel() * np.exp(0.5 * np.einsum("ij,ij->i", xx, xx)) * sig ** 3
    u = np.asarray(U, dtype=float)[None, :] + sig * xx
    return u, w


def total_temperature(T_inf: float, mach: float, gamma: float = 1.4) -> float:
    """Eq. 73: free-stream total temperature."""
    return T_inf * (1.0 + 0.5 * (gamma - 1.0) * mach * mach)


def refine_weight(T: float, R: float = 0.5) -> float:
    """Eq. 74: mean cell volume in a refined ball of radius 3*sqrt(R*T)."""
    r = 3.0 * math.sqrt(R * T)
    return (4.0 / 3.0) * math.pi * r ** 3 / (730.0 * (math.atan((T - 1.0) / 40.0) + 1.0))


def refine_count(T: float) -> float:
    """Number of velocity cells Eq. 74 puts in the refined ball of temperature T."""
    return 730.0 * (math.atan((T - 1.0) / 40.0) + 1.0)


def octree_dvs(center, radius: float, h_outer: float, refine=(), root_scale: float = 1.0):
    """Octree velocity mesh clipped to a ball.

    The bounding cube of the ball (edge 2*radius*root_scale) is split
    recursively.  A cube is split while its edge exceeds sqrt(2) times the
    target spacing (so leaf spacings land within a factor sqrt(2) of the
    target), which is ``h_outer`` away from the refinement balls and ``h``
    inside any ball (c, r, h) of ``refine`` that the cube touches.  Leaves whose
    centre lies in the outer ball are kept: the point is the cube centre (its
    centroid) and the weight its volume.
    """
    center = np.asarray(center, dtype=float)
    refine = [(np.asarray(c, dtype=float), float(r), float(h)) for c, r, h in refine]
    c = center[None, :].copy()
    s = 2.0 * radius * root_scale
    leaves_c, leaves_s = [], []
    octs = np.array([[dx, dy, dz] for dx in (-1, 1) for dy in (-1, 1) for dz in (-1, 1)], dtype=float)
    while len(c):
        d = np.maximum(np.abs(center[None, :] - c) - 0.5 * s, 0.0)
        c = c[np.einsum("ij,ij->i", d, d) <= radius * radius]
        target = np.full(len(c), float(h_outer))
        for bc, br, bh in refine:
            d = np.maximum(np.abs(bc[None, :] - c) - 0.5 * s, 0.0)
            touch = np.einsum("ij,ij->i", d, d) <= br * br
            target = np.where(touch, np.minimum(target, bh), target)
        split = s > target * math.sqrt(2.0)
        leaf = c[~split]
        keep = np.einsum("ij,ij->i", leaf - center, leaf - center) <= radius * radius
        leaves_c.append(leaf[keep])
        leaves_s.append(np.full(int(keep.sum()), s))
        c = (c[split][:, None, :] + 0.25 * s * octs[None, :, :]).reshape(-1, 3)
        s *= 0.5
    u = np.concatenate(leaves_c)
    w = np.concatenate(leaves_s) ** 3
    order = np.lexsort((u[:, 2], u[:, 1], u[:, 0]))
    return u[order], w[order]


def direction_order(u, bits: int = 5):
    """Permutation sorting velocities by direction, then by speed.

    Directions u/|u| are mapped to the plane by the octahedral projection and ordered along a Morton
    curve of 2^bits x 2^bits cells.  Consecutive velocities then point roughly the same way, so for any
    face normal the sign of u.n changes rarely along the set: whole wavefronts of the upwind kernels take
    the same branch and skip the same neighbour loads.  The order changes no result beyond rounding.
    """
    u = np.asarray(u, dtype=float)
    speed = np.linalg.norm(u, axis=1)
    d = u / np.maximum(speed, 1e-300)[:, None]
    l1 = np.maximum(np.abs(d).sum(axis=1), 1e-300)
    px, py = d[:, 0] / l1, d[:, 1] / l1
    lower = d[:, 2] < 0
    qx = np.where(lower, (1.0 - np.abs(py)) * np.sign(px), px)
    qy = np.where(lower, (1.0 - np.abs(px)) * np.sign(py), py)
    n = 1 << bits
    ix = np.clip(((qx + 1.0) * 0.5 * n).astype(np.int64), 0, n - 1)
    iy = np.clip(((qy + 1.0) * 0.5 * n).astype(np.int64), 0, n - 1)
    key = np.zeros(len(u), dtype=np.int64)
    for b in range(bits):
        key |= ((ix >> b) & 1) << (2 * b) | ((iy >> b) & 1) << (2 * b + 1)
    return np.lexsort((speed, key))


def paper_unstructured_dvs(U_inf, T_inf: float, T_w: float, mach: float, outer_radius_factor: float = 5.0,
                           h_outer: float = None, target: int = None, R: float = 0.5, gamma: float = 1.4,
                           refine_scale: float = 1.0):
    """Unstructured DVS following the empirical criterion of Sec. 4.4.

    Outer ball centred at 0.4*U_inf with radius outer_radius_factor*sqrt(R*max(T0, T_w)) (Eq. 73 for T0);
    refined balls of radius 3*sqrt(R*T) at U_inf (T = T_inf) and at 0 (T = T_w),
    with the mean weight of Eq. 74 giving their spacing (times ``refine_scale``, 1 by default;
    coarser sets for small tests).  ``h_outer`` (or a
    ``target`` total count, found by a small scan) sets the outer spacing.
    """
    U_inf = np.asarray(U_inf, dtype=float)
    T0 = total_temperature(T_inf, mach, gamma)
    radius = outer_radius_factor * math.sqrt(R * max(T0, T_w))
    refine = [(U_inf, 3.0 * math.sqrt(R * T_inf), refine_scale * refine_weight(T_inf, R) ** (1.0 / 3.0)),
              (np.zeros(3), 3.0 * math.sqrt(R * T_w), refine_scale * refine_weight(T_w, R) ** (1.0 / 3.0))]
    center = 0.4 * U_inf
    if h_outer is not None:
        u, w = octree_dvs(center, radius, h_outer, refine)
    else:
        # scan the root cube size and the outer level; keep the count closest to target
        best = None
        for scale in np.linspace(1.0, 1.95, 20):
            for lvl in range(2, 7):
                h = 2.0 * radius * scale / 2 ** lvl
                u, w = octree_dvs(center, radius, h, refine, root_scale=scale)
                if best is None or abs(len(u) - target) < abs(len(best[0]) - target):
                    best = (u, w)
        u, w = best
    o = direction_order(u)
    return u[o], w[o]
