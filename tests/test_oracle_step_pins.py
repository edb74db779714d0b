"""Pins of the oracle's reconstruction, limiter, flux assembly and macroscopic PR-SGS (no GPU).

Each test rebuilds one step of the oracle from its definition in the paper, with plain numpy on the oracle's
geometry, and compares:

* Venkatakrishnan's function (the limiter Eq. 46 cites) against its published closed-form values, and the
  minimum over a cell's faces against its value at the two extreme faces;
* the limiter of every cell against the minimum of that function over the cell's faces, evaluated by hand;
* the face value of Eq. 46 (the point x_f - u s, the upwind cell, the u.n = 0 tie) against a least-squares
  gradient taken with numpy's lstsq, on one face for every velocity;
* the micro (Eq. 31) and macro (Eq. 37) fluxes against the face fluxes they sum;
* the macroscopic increment of Eq. 43 against a dense solve (exact Jacobian mode), against the LU-SGS
  factorisation for one sweep pair, and, in the matrix-free mode, against the nonlinear equations it solves.
"""
import numpy as np
import pytest

import oracle
from paper_2303_10846_amd.cases import configs, dvs

R_GAS = 0.5


def rel(a, b):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------------------
# Venkatakrishnan's function (Eq. 46 limiter)
# ---------------------------------------------------------------------------

def venkat_ratio_form(y, e):
    """Venkatakrishnan's function in its published ratio form, y = d1/d2, e = eps^2/d2^2:
    (y^2 + 2y + e) / (y^2 + y + 2 + e)."""
    return (y * y + 2 * y + e) / (y * y + y + 2 + e)


def test_venkatakrishnan_function_published_values():
    psi = oracle.venkat_psi
    for d2 in (1e-3, 0.7, 5.0):
        # y = 1: 3/4; y = 2: exactly 1 (the point where the function first reaches 1); y = 0: 0
        assert abs(psi(d2, d2, 0.0) - 0.75) < 1e-15
        assert abs(psi(2 * d2, d2, 0.0) - 1.0) < 1e-15
        assert psi(0.0, d2, 0.0) == 0.0
        # the sign of (d1, d2) together does not matter (the min side mirrors the max side)
        assert abs(psi(-1.3 * d2, -d2, 0.0) - psi(1.3 * d2, d2, 0.0)) < 1e-15
    # no change towards the face: psi = 1
    assert psi(0.4, 0.0, 0.0) == 1.0
    # monotone increasing from 0 to 1 on y in [0, 2]
    ys = np.linspace(0.0, 2.0, 201)
    vals = np.array([psi(y, 1.0, 0.0) for y in ys])
    assert np.all(np.diff(vals) > 0) and vals[0] == 0.0 and abs(vals[-1] - 1.0) < 1e-15
    # the ratio form with the smoothing term, and eps -> infinity switches the limiter off
    for y, d2, eps2 in ((0.3, 0.2, 0.01), (1.7, -0.5, 0.3), (-0.4, 1.1, 2.0), (0.05, 3.0, 0.0)):
        assert abs(psi(y * d2, d2, eps2) - venkat_ratio_form(y, eps2 / d2 ** 2)) < 1e-14
    assert abs(psi(0.0, 1.0, 1e12) - 1.0) < 1e-11


def test_limiter_minimum_over_faces_is_at_the_two_extreme_faces():
    """min(1, min_f psi(d1_f, d2_f)) with d1_f = d_max (>= 0) where d2_f > 0 and d_min (<= 0) where d2_f < 0
    equals min(1, psi(d_max, max_f d2_f), psi(d_min, min_f d2_f)), each term taken only for a positive maximum or a
    negative minimum: for fixed d1 >= 0, min(1, psi) does not grow with d2 > 0 (psi < 1 exactly for d2 > d1/2,
    where it decreases), and the same with every sign reversed.  The reconstruction kernels evaluate the
    limiter at those two faces only; this checks the identity on the oracle's function, over random stencils
    with 1 to 6 faces, zero increments and eps = 0 included."""
    psi = oracle.venkat_psi
    rng = np.random.default_rng(11)

    def lim_all(dmax, dmin, d2, eps2):
        L = 1.0
        for x in d2:
            if x != 0.0:
                L = min(L, psi(dmax if x > 0 else dmin, x, eps2))
        return L

    def lim_two(dmax, dmin, d2, eps2):
        L = 1.0
        if max(d2) > 0:
            L = min(L, psi(dmax, max(d2), eps2))
        if min(d2) < 0:
            L = min(L, psi(dmin, min(d2), eps2))
        return L

    n_active = 0
    for t in range(4000):
        nf = int(rng.integers(1, 7))
        scale = 10.0 ** rng.uniform(-3, 1)
        d2 = list(scale * rng.normal(size=nf))
        for a in range(nf):
            if rng.uniform() < 0.15:
                d2[a] = 0.0
        dmax = 0.0 if rng.uniform() < 0.1 else abs(scale * rng.normal())
        dmin = 0.0 if rng.uniform() < 0.1 else -abs(scale * rng.normal())
        eps2 = 0.0 if rng.uniform() < 0.3 else (scale * 10.0 ** rng.uniform(-3, 0)) ** 2
        la, lt = lim_all(dmax, dmin, d2, eps2), lim_two(dmax, dmin, d2, eps2)
        assert abs(la - lt) <= 1e-15 * max(la, 1e-300), (dmax, dmin, d2, eps2, la, lt)
        n_active += la < 0.999
    assert n_active > 1000  # the limiter acts in many of the samples


def _lsq_gradients(geo, phi):
    """Unweighted least-squares gradient per cell (reading A19): rows d = x_nb - x_i with difference
    phi_nb - phi_i over the interior faces, and d = x_f - x_i with a zero difference over the boundary faces.
    Solved with numpy's lstsq, per cell, for all velocities at once.  Returns [nc][nv][3]."""
    nc, nv = phi.shape
    out = np.empty((nc, nv, 3))
    for i in range(nc):
        rows, rhs = [], []
        for f in geo["cf"][i]:
            j = geo["fn"][f] if geo["fo"][f] == i else geo["fo"][f]
            if j >= 0:
                rows.append(geo["xc"][j] - geo["xc"][i])
                rhs.append(phi[j] - phi[i])
            else:
                rows.append(geo["xf"][f] - geo["xc"][i])
                rhs.append(np.zeros(nv))
        sol, *_ = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)
        out[i] = sol.T
    return out


def _random_state(o, c, seed, spread=0.2):
    """A positive, non-smooth state: the initial equilibrium with independent +-spread noise per value."""
    rng = np.random.default_rng(seed)
    o.init_equilibrium(c["W0"])
    G, R, W, q = o.get_state()
    G = G * (1.0 + spread * rng.uniform(-1, 1, G.shape))
    R = R * (1.0 + spread * rng.uniform(-1, 1, R.shape))
    return G, R, W, q


def test_limiter_is_the_minimum_of_venkatakrishnan_over_the_faces():
    """L_i,k = min(1, min_f psi(d1, d2; eps^2)) with d2 = grad . (x_f - x_i), d1 = max or min over the cell and
    its face neighbours minus phi_i (by the sign of d2), eps^2 = (K h)^3 max(|phi_max|, |phi_min|)^2 (reading
    A19), rebuilt by hand from the unlimited gradients and compared with the oracle's limited gradients."""
    c = configs.cavity_case(n=3, nv_side=4)
    K = 0.7
    o_on = oracle.Oracle(c, num=dict(c["num"], limiter=1, lim_K=K))
    o_off = oracle.Oracle(c, num=dict(c["num"], limiter=0))
    G, R, W, q = _random_state(o_on, c, seed=5)
    for o in (o_on, o_off):
        o.set_state(G, R, W, q)
        o.explicit()
    geo = o_on.geometry()
    gu = o_off.stage("gradG")
    gl = o_on.stage("gradG")
    # the unlimited gradient is the least-squares one
    assert rel(gu, _lsq_gradients(geo, G)) < 1e-12
    nc, nv = G.shape
    L = np.ones((nc, nv))
    n_active = 0
    for i in range(nc):
        nbrs = [geo["fn"][f] if geo["fo"][f] == i else geo["fo"][f] for f in geo["cf"][i]]
        nbrs = [j for j in nbrs if j >= 0]
        stencil = G[[i] + nbrs]
        pmax, pmin = stencil.max(axis=0), stencil.min(axis=0)
        eps2 = (K * geo["h"][i]) ** 3 * np.maximum(np.abs(pmax), np.abs(pmin)) ** 2
        for f in geo["cf"][i]:
            d2 = gu[i] @ (geo["xf"][f] - geo["xc"][i])
            d1 = np.where(d2 > 0, pmax - G[i], pmin - G[i])
            with np.errstate(divide="ignore", invalid="ignore"):
                psi = np.where(d2 != 0, venkat_ratio_form(d1 / d2, eps2 / d2 ** 2), 1.0)
            L[i] = np.minimum(L[i], psi)
        n_active += int(np.sum(L[i] < 0.999))
    assert n_active > nc * nv // 20  # the noise makes the limiter act on many (cell, velocity) pairs
    assert rel(gl, L[:, :, None] * gu) < 1e-12


# ---------------------------------------------------------------------------
# Eq. 46: the reconstruction point and the upwind cell, on one face, by hand
# ---------------------------------------------------------------------------

def _tie_case():
    """Cavity with a 4^3 Cartesian DVS plus one velocity lying exactly in the plane of one interior face
    (its u.n is zero up to rounding, so the tie rule of reading A11 picks cell j)."""
    c = configs.cavity_case(n=3, nv_side=4)
    o = oracle.Oracle(c)
    geo = o.geometry()
    interior = np.nonzero(geo["fn"] >= 0)[0]
    f_star = int(interior[len(interior) // 2])
    n = geo["n"][f_star]
    t = np.cross(n, np.array([0.3, 0.5, 0.8]))
    u_tie = 2.0 * t / np.linalg.norm(t)
    c["u"] = np.vstack([c["u"], u_tie])
    c["w"] = np.append(c["w"], c["w"][0])
    return c, f_star


def test_face_value_is_taken_at_x_f_minus_u_s_in_the_upwind_cell():
    """Free-molecular limit (tau -> infinity, so phi_f = phi_bar, Eq. 45): on one interior face, every velocity's
    A (u.n) phi_f equals A (u.n) [phi_c + (x_f - u s - x_c) . grad_c phi] with c = i for u.n > 0 and c = j
    otherwise (Eq. 46), the gradient from numpy's least squares; on a boundary face the outgoing velocities do
    the same from cell i."""
    c, f_star = _tie_case()
    gas = dict(c["gas"], mu_ref=1e18)
    o = oracle.Oracle(c, gas=gas, num=dict(c["num"], limiter=0))
    G, R, W, q = _random_state(o, c, seed=11)
    o.set_state(G, R, W, q)
    o.explicit()
    geo = o.geometry()
    gG = _lsq_gradients(geo, G)
    u = c["u"]
    ffG = o.stage("ffG")
    checked = 0
    for f in [f_star] + [int(x) for x in np.nonzero(geo["fn"] < 0)[0][:3]]:
        i, j, n, s, A = geo["fo"][f], geo["fn"][f], geo["n"][f], geo["s"][f], geo["A"][f]
        un = u @ n
        for k in range(len(u)):
            if abs(un[k]) <= 1e-13 * np.linalg.norm(u[k]):
                continue  # no flux through the face at u.n = 0
            if un[k] <= 0 and j < 0:
                continue  # boundary ghost side
            cc = i if un[k] > 0 else j
            xp = geo["xf"][f] - u[k] * s
            phibar = G[cc, k] + (xp - geo["xc"][cc]) @ gG[cc, k]
            want = A * un[k] * phibar
            assert abs(ffG[f, k] - want) <= 1e-12 * abs(want), (f, k)
            checked += 1
    assert checked > 60


def test_face_collision_uses_the_tie_velocity_from_cell_j():
    """Finite tau: the face distribution of one interior face is the Eq. 45 collision step applied to the face
    values of Eq. 46 for all velocities, including the one with u.n = 0, which comes from cell j (reading A11).
    Taking it from cell i instead changes the face moments and every face value."""
    c, f_star = _tie_case()
    o = oracle.Oracle(c, num=dict(c["num"], limiter=0))
    G, R, W, q = _random_state(o, c, seed=12)
    o.set_state(G, R, W, q)
    o.explicit()
    geo = o.geometry()
    gG, gR = _lsq_gradients(geo, G), _lsq_gradients(geo, R)
    u, w = c["u"], c["w"]
    f = f_star
    i, j, n, s, A = geo["fo"][f], geo["fn"][f], geo["n"][f], geo["s"][f], geo["A"][f]
    un = u @ n
    tie = np.abs(un) <= 1e-13 * np.linalg.norm(u, axis=1)
    assert tie.sum() == 1 and tie[-1]

    def phibar(side_of_tie):
        cc = np.where(un > 0, i, j)
        cc[tie] = side_of_tie
        xp = geo["xf"][f][None, :] - u * s - geo["xc"][cc]
        Gb = G[cc, np.arange(len(u))] + np.einsum("kd,kd->k", xp, gG[cc, np.arange(len(u))])
        Rb = R[cc, np.arange(len(u))] + np.einsum("kd,kd->k", xp, gR[cc, np.arange(len(u))])
        return Gb, Rb

    ffG = o.stage("ffG")[f]
    Gb, Rb = phibar(j)
    Gf, _, _ = oracle.face_collision(u, w, Gb, Rb, s, c["gas"])
    assert rel(ffG[~tie], A * un[~tie] * Gf[~tie]) < 1e-12
    Gb_i, Rb_i = phibar(i)
    Gf_i, _, _ = oracle.face_collision(u, w, Gb_i, Rb_i, s, c["gas"])
    assert rel(ffG[~tie], A * un[~tie] * Gf_i[~tie]) > 1e-8


def test_micro_and_macro_fluxes_are_the_signed_sums_of_the_face_fluxes():
    """Eq. 31: F_i,k = (1/V_i) sum_f (+-) A_f (u.n_f) phi_f,k, the sign + where n_f points out of cell i.
    Eq. 37: the macro face flux is the DVS moment sum_k w_k Phi_k of the micro face flux, and F_i sums it the
    same way."""
    c = configs.open_box_case(n=2, nv_side=5)
    o = oracle.Oracle(c)
    o.init_equilibrium(c["W0"])
    o.iterate(2)
    o.explicit()
    geo = o.geometry()
    u, w = c["u"], c["w"]
    ffG, ffR, ffmac = o.stage("ffG"), o.stage("ffR"), o.stage("ffmac")
    FG, FR, Fmac = o.stage("FG"), o.stage("FR"), o.stage("Fmac")
    u2 = 0.5 * np.sum(u * u, axis=1)
    mom = np.stack([ffG @ w, (ffG * w) @ u[:, 0], (ffG * w) @ u[:, 1], (ffG * w) @ u[:, 2],
                    (ffG * w) @ u2 + ffR @ w, ffR @ w], axis=1)
    assert rel(ffmac, mom) < 1e-13
    nc = o.nc
    FG_h, FR_h, Fm_h = np.zeros_like(FG), np.zeros_like(FR), np.zeros((nc, 6))
    for f in range(o.nf):
        for cell, sg in ((geo["fo"][f], 1.0), (geo["fn"][f], -1.0)):
            if cell < 0:
                continue
            FG_h[cell] += sg * ffG[f] / geo["V"][cell]
            FR_h[cell] += sg * ffR[f] / geo["V"][cell]
            Fm_h[cell] += sg * ffmac[f] / geo["V"][cell]
    assert rel(FG, FG_h) < 1e-13 and rel(FR, FR_h) < 1e-13 and rel(Fmac, Fm_h) < 1e-13


# ---------------------------------------------------------------------------
# Eqs. 38-43: the macroscopic system, assembled densely by hand
# ---------------------------------------------------------------------------

def euler_flux_np(W, n, R=R_GAS):
    """Euler flux of Eq. 40 with the rotational-energy row; p = rho R T with 5 degrees of freedom, so
    p = (2/5)(rho E - rho |U|^2 / 2).  Works on complex W (complex-step Jacobians)."""
    rho = W[0]
    U = W[1:4] / rho
    p = 0.4 * (W[4] - 0.5 * rho * np.sum(U * U))
    Un = np.sum(U * n)
    return np.array([rho * Un, W[1] * Un + p * n[0], W[2] * Un + p * n[1], W[3] * Un + p * n[2],
                     (W[4] + p) * Un, W[5] * Un])


def euler_jacobian(W, n):
    """dG/dW by complex step (exact to rounding)."""
    J = np.empty((6, 6))
    h = 1e-30
    for m in range(6):
        Wc = W.astype(complex)
        Wc[m] += 1j * h
        J[:, m] = euler_flux_np(Wc, n).imag / h
    return J


def primitives_np(W, R=R_GAS):
    rho = W[:, 0]
    U = W[:, 1:4] / rho[:, None]
    ke = 0.5 * rho * np.sum(U * U, axis=1)
    T = 0.4 * (W[:, 4] - ke) / (rho * R)
    Ttr = (2.0 / 3.0) * (W[:, 4] - ke - W[:, 5]) / (rho * R)
    return rho, U, T, Ttr


def macro_system(o, c, W, Fmac):
    """Dense Eq. 43 system M dW = b over the 6 N unknowns: diagonal blocks D_i (1/dt + (1/2) sum_f (A/V_i) r_f,
    plus 1/(Z tau_i) in the rho E_rot row), off-diagonal blocks (1/2)(A/V_i)(dG/dW(W_j) - r_f I) with the normal
    out of cell i, right-hand side -F_i plus the rotational source (rho R T - rho E_rot)/(Z tau) (readings A12,
    A13: face state = mean of the two cells, lagged source)."""
    geo = o.geometry()
    gas, num = c["gas"], o.num
    nc = o.nc
    rho, U, T, Ttr = primitives_np(W)
    mu = lambda t: gas["mu_ref"] * (t / gas["T_ref"]) ** gas["omega_vhs"]
    tau = mu(Ttr) / (rho * R_GAS * Ttr)
    umax = np.max(np.linalg.norm(c["u"], axis=1))
    inv_dt = num["inv_dt"] + (umax / (num["cfl_imp"] * geo["h"]) if num["cfl_imp"] > 0 else 0.0)
    M = np.zeros((6 * nc, 6 * nc))
    b = np.zeros(6 * nc)
    rfs = np.zeros(o.nf)
    diag = np.broadcast_to(inv_dt, (nc,)).astype(float).copy()
    for f in range(o.nf):
        i, j = geo["fo"][f], geo["fn"][f]
        jj = j if j >= 0 else i
        rf, Tf, Ttrf = 0.5 * (rho[i] + rho[jj]), 0.5 * (T[i] + T[jj]), 0.5 * (Ttr[i] + Ttr[jj])
        Unf = 0.5 * (U[i] + U[jj]) @ geo["n"][f]
        dl = np.linalg.norm(geo["xc"][i] - geo["xc"][j]) if j >= 0 else 2 * np.linalg.norm(geo["xf"][f] - geo["xc"][i])
        r = abs(Unf) + np.sqrt(gas["gamma"] * R_GAS * Tf) + 2 * mu(Ttrf) / (rf * dl)
        rfs[f] = r
        for a, bb, sg in ((i, j, 1.0), (j, i, -1.0)):
            if a < 0:
                continue
            av = geo["A"][f] / geo["V"][a]
            diag[a] += 0.5 * av * r
            if bb >= 0:
                Jn = euler_jacobian(W[bb], sg * geo["n"][f])
                M[6 * a:6 * a + 6, 6 * bb:6 * bb + 6] += 0.5 * av * (Jn - r * np.eye(6))
    for i in range(nc):
        M[6 * i:6 * i + 6, 6 * i:6 * i + 6] += diag[i] * np.eye(6)
        M[6 * i + 5, 6 * i + 5] += 1.0 / (gas["Z"] * tau[i])
        b[6 * i:6 * i + 6] = -Fmac[i]
        b[6 * i + 5] += (rho[i] * R_GAS * T[i] - W[i, 5]) / (gas["Z"] * tau[i])
    return M, b, rfs


def _macro_case(**num):
    c = configs.cavity_case(n=2, nv_side=4, lid_speed=0.3)
    c["num"] = dict(c["num"], cfl_imp=2.0, **num)
    o = oracle.Oracle(c)
    o.init_equilibrium(c["W0"])
    o.iterate(4)                   # a non-uniform W with flow
    _, _, W, _ = o.get_state()
    o.iterate(1)
    return c, o, W


def test_macro_pr_sgs_converges_to_the_dense_solve_of_eq43():
    c, o, W = _macro_case(macro_exact_jvp=1, n_macro=400)
    M, b, _ = macro_system(o, c, W, o.stage("Fmac"))
    x = np.linalg.solve(M, b).reshape(-1, 6)
    dW = o.stage("dW")
    assert np.max(np.abs(x)) > 1e-4
    assert rel(dW, x) < 1e-11
    assert rel(o.stage("Wt"), W + x) < 1e-13


def test_one_macro_sweep_pair_is_the_block_lu_sgs_step():
    """With one forward + backward pair from zero, the increment solves (D + L) D^-1 (D + U) dW = b with the
    6x6 blocks of the dense system split in the sweep (cell) order."""
    c, o, W = _macro_case(macro_exact_jvp=1, n_macro=1)
    M, b, _ = macro_system(o, c, W, o.stage("Fmac"))
    nc = o.nc
    D = np.zeros_like(M)
    for i in range(nc):
        D[6 * i:6 * i + 6, 6 * i:6 * i + 6] = M[6 * i:6 * i + 6, 6 * i:6 * i + 6]
    blk = np.kron(np.arange(nc), np.ones(6, dtype=int))
    L = np.where(blk[:, None] > blk[None, :], M, 0.0)
    U = np.where(blk[:, None] < blk[None, :], M, 0.0)
    y = np.linalg.solve(D + L, b)
    x = np.linalg.solve(D + U, D @ y).reshape(-1, 6)
    assert rel(o.stage("dW"), x) < 1e-11
    assert rel(o.stage("dW"), np.linalg.solve(M, b).reshape(-1, 6)) > 1e-6


def test_matrix_free_macro_increment_solves_the_nonlinear_eq43():
    """Default mode (reading A14): dG_j = G(W_j + dW_j) - G(W_j).  After many pairs the increment satisfies
    D_i dW_i + sum_j (1/2)(A/V_i)[G(W_j + dW_j) - G(W_j) - r_f dW_j] = b_i at every cell."""
    c, o, W = _macro_case(macro_exact_jvp=0, n_macro=400)
    Fmac = o.stage("Fmac")
    dW = o.stage("dW")
    M, b, rfs = macro_system(o, c, W, Fmac)
    geo = o.geometry()
    nc = o.nc
    lhs = np.zeros((nc, 6))
    for i in range(nc):
        lhs[i] = M[6 * i:6 * i + 6, 6 * i:6 * i + 6] @ dW[i]
    # off-diagonal part, evaluated with the nonlinear flux difference in place of the Jacobian
    for f in range(o.nf):
        i, j = geo["fo"][f], geo["fn"][f]
        if j < 0:
            continue
        for a, bb, sg in ((i, j, 1.0), (j, i, -1.0)):
            n = sg * geo["n"][f]
            av = geo["A"][f] / geo["V"][a]
            dG = euler_flux_np(W[bb] + dW[bb], n) - euler_flux_np(W[bb], n)
            lhs[a] += 0.5 * av * (dG - rfs[f] * dW[bb])
    assert np.max(np.abs(dW)) > 1e-4
    assert rel(lhs, b.reshape(-1, 6)) < 1e-11
    # and it differs from the linear (exact Jacobian) solve by the second-order flux terms only
    x = np.linalg.solve(M, b).reshape(-1, 6)
    assert 1e-12 < rel(dW, x) < 1e-2


# ---------------------------------------------------------------------------
# Limiter freezing (limiter = 3): stored Venkatakrishnan values in place of the limiter
# ---------------------------------------------------------------------------

def test_frozen_limiter_reuses_the_values_of_the_state_it_was_frozen_at():
    """At the state it was frozen at, limiter 3 reconstructs exactly as limiter 1; at another state it scales the
    unlimited least-squares gradient by the stored values, not by the limiter of the new state."""
    c = configs.cavity_case(n=3, nv_side=4)
    o1 = oracle.Oracle(c, num=dict(c["num"], limiter=1))
    o3 = oracle.Oracle(c, num=dict(c["num"], limiter=1))
    o0 = oracle.Oracle(c, num=dict(c["num"], limiter=0))
    G, R, W, q = _random_state(o1, c, seed=21)
    for o in (o1, o3):
        o.set_state(G, R, W, q)
    o3.freeze_limiter()
    o1.explicit()
    o3.explicit()
    for st in ("gradG", "gradR", "FG", "FR", "Fmac"):
        assert np.array_equal(o1.stage(st), o3.stage(st)), st
    # the stored values, recovered from the limited and unlimited gradients at the freezing state
    o0.set_state(G, R, W, q)
    o0.explicit()
    gu, gl = o0.stage("gradG"), o1.stage("gradG")
    nz = np.abs(gu) > 1e-10 * np.abs(gu).max()
    Lg = np.where(nz[..., 0], gl[..., 0] / np.where(nz[..., 0], gu[..., 0], 1.0), 1.0)
    assert Lg.min() < 0.9
    # another state: limiter 3 keeps the stored values
    rng = np.random.default_rng(22)
    G2 = G * (1.0 + 0.1 * rng.uniform(-1, 1, G.shape))
    for o in (o0, o1, o3):
        o.set_state(G2, R, W, q)
        o.explicit()
    gu2, gl2, g3 = o0.stage("gradG"), o1.stage("gradG"), o3.stage("gradG")
    assert rel(g3[nz[..., 0]], (Lg[..., None] * gu2)[nz[..., 0]]) < 1e-12
    assert rel(g3, gl2) > 1e-3   # the recomputed limiter would differ


def test_frozen_limiter_scheme_is_smooth_complex_step_matches_central_differences():
    """With the limiter values frozen the steady residual is a smooth function of the state: its complex-step
    derivative along a random direction matches central differences to the truncation error."""
    c = configs.open_box_case(n=2, nv_side=5)
    o = oracle.Oracle(c, num=dict(c["num"], limiter=1))
    o.init_equilibrium(c["W0"])
    o.iterate(6)
    o.freeze_limiter()
    G, R, W, q = o.get_state()
    rng = np.random.default_rng(23)
    u = [rng.standard_normal(x.shape) * np.abs(x).max() for x in (G, R, W, q)]
    up = np.zeros(3)
    jG, jR, jW, jq, jJ = o.steady_residual_jvp(*u, up)
    h = 1e-6
    outs = []
    for sg in (1.0, -1.0):
        o.set_state(*[x + sg * h * du for x, du in zip((G, R, W, q), u)])
        outs.append(o.steady_residual(1))
    o.set_state(G, R, W, q)
    for m, jx in enumerate((jG, jR, jW, jq)):
        fd = (outs[0][m] - outs[1][m]) / (2 * h)
        assert rel(jx, fd) < 1e-6, m
    assert abs(jJ - (outs[0][4] - outs[1][4]) / (2 * h)) <= 1e-6 * abs(jJ)
