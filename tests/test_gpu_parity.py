"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Metric: for an array a against the oracle's b, max|a - b| / max|b| per field
(per component for W and q).  Bar for the FP64 path: 1e-11.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2303_10846_amd.cases import configs

pytestmark = pytest.mark.gpu

TOL = 1e-11


def nrel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def colrel(a, b):
    """nrel per column.  A column whose largest value is below 1e-6 of the whole array's is zero by an identity
    up to the rounding of terms as large as the other columns (e.g. the mass flux of a cell closed by walls,
    which cancels to zero), so it is measured against the whole array's largest value."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    top = float(np.max(np.abs(b)))
    out = 0.0
    for m in range(a.shape[1]):
        col = float(np.max(np.abs(b[:, m])))
        scale = col if col >= 1e-6 * top else top
        out = max(out, float(np.max(np.abs(a[:, m] - b[:, m]))) / max(scale, 1e-300))
    return out


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def solver(case, precision="fp64", num=None):
    from paper_2303_10846_amd.binding import Solver
    return Solver(case, precision=precision, num=num)


def _pair(case, warm=3, num=None):
    """Oracle and GPU solver on the same case, both set to the oracle's state after `warm` iterations."""
    o = oracle.Oracle(case, num=num)
    o.init_equilibrium(case["W0"])
    if warm:
        o.iterate(warm)
    G, R, W, q = o.get_state()
    s = solver(case, num=num)
    s.set_state(G, R, W, q)
    return o, s


def _tets_case(n):
    """Degenerate meshes: one tetrahedron with four wall faces, or two sharing one face (one interior face,
    two colours).  The tag-2 face is a moving hot wall."""
    from paper_2303_10846_amd.cases import dvs, mesh
    xyz = 0.5 * np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], dtype=float)[:3 + n]
    tets = mesh._orient(xyz, np.array([[0, 1, 2, 3], [1, 2, 3, 4]])[:n])
    tets_c, off = mesh.color_major(xyz, tets)
    btri = mesh.boundary_triangles(tets_c)
    btag = np.ones(len(btri), dtype=np.int64)
    btag[0] = 2
    u, w = dvs.cartesian_dvs(6, 4.0)
    bcs = [configs._bc(1, configs.WALL, T=1.0), configs._bc(2, configs.WALL, U=(0.1, 0.0, 0.0), T=1.5)]
    return dict(name=f"tets{n}", mesh=dict(xyz=xyz, tets=tets_c, btri=btri, btag=btag, color_offsets=off), u=u,
                w=w, gas=configs.gas_n2(0.1, 3.0), num=configs.numerics_default(), bcs=bcs, W0=configs.rest_state())


CASES = {
    "one_tet": lambda: _tets_case(1),                                       # a single cell, every face a wall
    "two_tets": lambda: _tets_case(2),                                      # one interior face
    "cavity_n2_dvs4": lambda: configs.cavity_case(n=2, nv_side=4),          # nv = 64 < one workgroup
    "cavity_n3_dvs7": lambda: configs.cavity_case(n=3, nv_side=7),          # nv = 343, ragged tail
    "open_box_n3": lambda: configs.open_box_case(n=3, nv_side=6),           # far field + hot wall
    "small_sphere": lambda: configs.small_sphere_case(),                    # unstructured DVS, 1944 tets
    "small_sphere_sutherland": lambda: _sutherland(configs.small_sphere_case(), 0.5),   # Eq. 14 viscosity
    "hex_cavity_n3_dvs6": lambda: configs.cavity_case(n=3, nv_side=6, kind="hex"),        # warped hexahedra
    "mixed_box_n4_dvs5": lambda: configs.open_box_case(n=4, nv_side=5, kind="mixed"),     # hex + pyramid + tet
    "small_sphere_hex": lambda: configs.small_sphere_hex_case(),                          # graded hex O-grid
}


def _sutherland(case, C_s):
    case["gas"] = dict(case["gas"], C_s=C_s)
    return case


@pytest.mark.parametrize("name", list(CASES))
def test_explicit_operator_fp64(name):
    say("case", name)
    c = CASES[name]()
    o, s = _pair(c)
    o.explicit()
    FG, FR, Fm = s.residual()
    assert nrel(FG.cpu().numpy(), o.stage("FG")) < TOL
    assert nrel(FR.cpu().numpy(), o.stage("FR")) < TOL
    assert colrel(Fm, o.stage("Fmac")) < TOL


@pytest.mark.parametrize("name", list(CASES))
def test_one_iteration_stage_by_stage_fp64(name):
    say("case", name)
    c = CASES[name]()
    o, s = _pair(c)
    ho = o.iterate(1)
    hs = s.iterate(1)
    assert colrel(s.debug_stage("dW"), o.stage("dW")) < TOL          # Eq. 43 (40 PR-SGS sweeps)
    assert colrel(s.debug_stage("Wt"), o.stage("Wt")) < TOL
    assert nrel(s.debug_stage("tau_t"), o.stage("tau_t")) < TOL
    assert nrel(s.resG.cpu().numpy(), o.stage("ResG")) < TOL          # Eq. 33 right-hand side
    assert nrel(s.resR.cpu().numpy(), o.stage("ResR")) < TOL
    assert nrel(s.dG.cpu().numpy(), o.stage("dG")) < TOL              # 2 PR-SGS sweeps of Eq. 33
    assert nrel(s.dR.cpu().numpy(), o.stage("dR")) < TOL
    G, R, W, q = s.get_state()
    Go, Ro, Wo, qo = o.get_state()
    assert nrel(G, Go) < TOL and nrel(R, Ro) < TOL
    assert colrel(W, Wo) < TOL                                        # Eqs. 62-65
    assert colrel(q, qo) < 1e-10                                      # Eqs. 66-67 (small, cancelling sums)
    assert np.max(np.abs(hs - ho)) <= 1e-11 * np.max(np.abs(ho)) + 1e-20


@pytest.mark.parametrize("kind", ["hex", "mixed"])
def test_hex_and_mixed_meshes_ten_iterations(kind):
    """Hexahedral and mixed meshes (6 face slots, 16-bit upwind codes): ten iterations from rest in FP64 against
    the oracle to 1e-11, and in the mixed precision (vector kernels with 16-bit codes, nv = 216) to FP32
    rounding; the upwind codes against the oracle's decisions slot by slot.  The mixed bar is that of the tet
    cavity (nearly at rest, Res cancels by ~1e3: measured 3.2e-5 on the hex cavity) and 1e-5 on the open box
    with flow."""
    c = configs.cavity_case(n=3, nv_side=6, kind=kind) if kind == "hex" else configs.open_box_case(
        n=4, nv_side=6, kind="mixed")
    say("case", c["name"])
    o = oracle.Oracle(c)
    o.init_equilibrium(c["W0"])
    ho = o.iterate(10)
    s = solver(c)
    s.init_equilibrium(c["W0"])
    hs = s.iterate(10)
    G, R, W, q = s.get_state()
    Go, Ro, Wo, qo = o.get_state()
    assert nrel(G, Go) < TOL and nrel(R, Ro) < TOL and colrel(W, Wo) < TOL
    assert np.max(np.abs(hs - ho)) <= 1e-11 * np.max(np.abs(ho))
    # upwind codes, 2 bits per slot in the slot order of the cell kind (unused slots 0)
    g = o.geometry()
    codes = s.upwind.cpu().numpy().astype(np.int64) & 0xFFFF
    u = np.asarray(c["u"], dtype=np.float64)
    snap = c["num"]["snap"] * np.linalg.norm(u, axis=1)
    want = np.zeros_like(codes)
    nc = codes.shape[0]
    for a in range(g["cf"].shape[1]):
        f = g["cf"][:, a]
        ok = f >= 0
        fs = np.where(ok, f, 0)
        sign = np.where(g["fo"][fs] == np.arange(nc), 1.0, -1.0)
        un = (u @ g["n"][fs].T).T * sign[:, None]
        ca = np.where(un > snap[None, :], 1, np.where(un < -snap[None, :], 2, 0)) * ok[:, None]
        want |= ca << (2 * a)
    assert np.array_equal(codes, want)
    sm = solver(c, precision="mixed")
    sm.init_equilibrium(c["W0"])
    sm.iterate(10)
    Wm, _ = sm.moments()
    eW = colrel(Wm, Wo)
    say(f"mixed precision after 10 iterations: W {eW:.2e}")
    assert eW < (1e-4 if kind == "hex" else 1e-5)


def test_frozen_limiter_values_fp64():
    """Limiter freezing (limiter 3): the values stored by cis_limiter_freeze equal the limiter of the state they
    were taken at, so the explicit operator there is that of limiter 1; on a later state they stay fixed, and the
    GPU iteration with them matches the oracle's frozen iteration."""
    say("case open box frozen limiter")
    c = configs.open_box_case(n=3, nv_side=6)
    o, s = _pair(c, warm=4)
    FG1, FR1, Fm1 = s.residual()
    o.freeze_limiter()
    L = s.freeze_limiter().cpu().numpy()
    assert 0.0 <= L.min() < 0.9 and L.max() <= 1.0
    FG3, FR3, Fm3 = s.residual()
    assert np.array_equal(FG1.cpu().numpy(), FG3.cpu().numpy()) and np.array_equal(Fm1, Fm3)
    o.iterate(5)
    s.iterate(5)
    Go, Ro, Wo, qo = o.get_state()
    Gs, Rs, Ws, qs = s.get_state()
    assert nrel(Gs, Go) < TOL and nrel(Rs, Ro) < TOL and colrel(Ws, Wo) < TOL and colrel(qs, qo) < TOL
    o.explicit()
    FG, _, Fm = s.residual()
    assert nrel(FG.cpu().numpy(), o.stage("FG")) < TOL and colrel(Fm, o.stage("Fmac")) < TOL
    # the stored values did not move, and detaching them is refused while limiter 3 is in use
    assert np.array_equal(s.L_frozen.cpu().numpy(), L)
    assert s.lib.cis_limiter_freeze(s.h, None, 0) == -1
    s.unfreeze_limiter()
    assert s.num["limiter"] == 1


def test_lu_sgs_settings_one_pair_each_fp64():
    """LU-SGS for both implicit systems: one forward + backward pair from zero (n_macro = n_micro = 1), which for
    Eq. 33 is the LU-SGS step (D + L) D^-1 (D + U) dphi = Res; stage-by-stage against the oracle."""
    c = configs.small_sphere_case()
    say("case", c["name"], "n_macro = n_micro = 1")
    num = dict(c["num"], n_macro=1, n_micro=1)
    o, s = _pair(c, warm=3, num=num)
    o.iterate(1)
    s.iterate(1)
    assert colrel(s.debug_stage("dW"), o.stage("dW")) < TOL
    assert nrel(s.dG.cpu().numpy(), o.stage("dG")) < TOL
    assert nrel(s.dR.cpu().numpy(), o.stage("dR")) < TOL
    G, R, W, q = s.get_state()
    Go, Ro, Wo, qo = o.get_state()
    assert nrel(G, Go) < TOL and colrel(W, Wo) < TOL and colrel(q, qo) < 1e-10


def test_cavity_full_config_200_iterations_fp64():
    """The 6x6x6x6-tet cavity with the 8^3 DVS (1296 x 512), 200 iterations from rest."""
    c = configs.cavity_case(seed=0)
    say("case", c["name"])
    o = oracle.Oracle(c)
    o.init_equilibrium(c["W0"])
    s = solver(c)
    s.init_equilibrium(c["W0"])
    for n in (1, 9, 190):
        ho = o.iterate(n)
        hs = s.iterate(n)
        _, _, Wo, _ = o.get_state()
        W, _ = s.moments()
        e = colrel(W, Wo)
        say(f"after {n} more iterations: W parity {e:.2e}, residual gpu {hs[-1].max():.2e} oracle {ho[-1].max():.2e}")
        assert e < TOL
    assert hs[-1].max() < 1e-13
    ql, qw = s.wall_heat_flux(2), s.wall_heat_flux(1)
    assert abs(ql - o.wall_heat_flux(2)) < 1e-11 * abs(ql)
    assert abs(ql + qw) < 1e-10 * abs(ql)


def test_small_sphere_from_rest_ten_iterations_fp64():
    c = configs.small_sphere_case()
    o = oracle.Oracle(c)
    o.init_equilibrium(c["W0"])
    s = solver(c)
    s.init_equilibrium(c["W0"])
    ho = o.iterate(10)
    hs = s.iterate(10)
    _, _, Wo, qo = o.get_state()
    W, q = s.moments()
    assert colrel(W, Wo) < TOL
    assert colrel(q, qo) < 1e-10
    assert np.max(np.abs(hs - ho) / np.maximum(np.abs(ho), 1e-300)) < 1e-9
    assert abs(s.wall_heat_flux(1) - o.wall_heat_flux(1)) < 1e-11 * abs(o.wall_heat_flux(1))


@pytest.mark.parametrize("nv_side", [17, 18])
def test_large_dvs_face_staging_paths_fp64(nv_side):
    """The FP64 face kernel's wide and prefix staging: nv = 17^3 = 4 913 stages both rows (77 KB) in one
    512-thread workgroup by ordinary loads (nv not a multiple of 4); nv = 18^3 = 5 832 (two rows of 46 KB) stages
    the first 2 304 velocities of G and R and re-reads the rest from global memory, as nv = 16 384 does
    (test_maximum_velocity_count).  The full sphere's FP64 rows (33 KB) take LDS-DMA in 512-thread workgroups,
    nv = 343 stages both rows without LDS-DMA in 256 threads, and the other cases take LDS-DMA in 256 threads."""
    c = configs.cavity_case(n=2, nv_side=nv_side)
    o, s = _pair(c, warm=2)
    o.iterate(1)
    s.iterate(1)
    G, R, W, q = s.get_state()
    Go, Ro, Wo, qo = o.get_state()
    assert nrel(G, Go) < TOL and colrel(W, Wo) < TOL


@pytest.mark.parametrize("nv_side", [7, 17, 18, 22])
def test_face_staging_paths_mixed(nv_side):
    """The mixed face kernel's staging paths against the FP64 oracle: nv = 343 stages G and R in LDS by ordinary
    loads in 256 threads (nv not a multiple of 4, so no LDS-DMA), nv = 4 913 the same in 512 threads (the pair is
    38.4 KB, over the 38 KB of a 256-thread workgroup), nv = 5 832 stages G, R and the codes by LDS-DMA in 512
    threads (51 KB), nv = 10 648 stages the first 4 864 velocities of G and R (the pair is 83 KB, over the 77 KB
    of a 512-thread workgroup); the 256-thread LDS-DMA path is that of every other mixed case.  Both sides start from the same FP32-rounded state three iterations from rest.  The cavity's cell fluxes
    are sums of face fluxes that nearly cancel, and each face's macro flux a velocity sum that nearly cancels,
    so the error is measured against the sums of the absolute terms: sum_f |A (u.n) phi_f| / V per (cell,
    velocity), and sum_f sum_k w |Psi_k| |A (u.n) phi_f,k| / V per cell and macro-flux column (Psi = 1, |u_x|,
    |u_y|, |u_z|, |u|^2/2 for G with 1 for R, 1 for R): FP32 rounding of those terms, some units of 6e-8
    (bar 1e-6); a wrong staged value gives errors of order one."""
    say("case cavity n2 mixed face staging nv_side", nv_side)
    c = configs.cavity_case(n=2, nv_side=nv_side)
    o = oracle.Oracle(c)
    o.init_equilibrium(c["W0"])
    o.iterate(3)
    G, R, W, q = o.get_state()
    G32, R32 = G.astype(np.float32), R.astype(np.float32)
    o.set_state(G32.astype(np.float64), R32.astype(np.float64), W, q)
    s = solver(c, precision="mixed")
    s.set_state(G32, R32, W, q)
    FG, FR, Fm = s.residual()
    o.explicit()
    g = o.geometry()
    cf, V = g["cf"], g["V"]

    def terms(ff):
        """sum over each cell's faces of |ff[face]| / V"""
        t = np.zeros((o.nc,) + ff.shape[1:])
        for a in range(cf.shape[1]):
            ok = cf[:, a] >= 0
            t[ok] += np.abs(ff[cf[ok, a]])
        return t / V.reshape((-1,) + (1,) * (ff.ndim - 1))

    eF = max(float(np.max(np.abs(FG.cpu().numpy() - o.stage("FG")))) / float(np.max(terms(o.stage("ffG")))),
             float(np.max(np.abs(FR.cpu().numpy() - o.stage("FR")))) / float(np.max(terms(o.stage("ffR")))))
    aG, aR = np.abs(o.stage("ffG")), np.abs(o.stage("ffR"))
    u, wq = np.asarray(c["u"]), np.asarray(c["w"])
    fmac_terms = np.stack([aG @ wq, aG @ (wq * np.abs(u[:, 0])), aG @ (wq * np.abs(u[:, 1])),
                           aG @ (wq * np.abs(u[:, 2])), aG @ (0.5 * wq * np.sum(u * u, axis=1)) + aR @ wq,
                           aR @ wq], axis=1)
    tm = np.max(terms(fmac_terms), axis=0)
    eFm = float(np.max(np.max(np.abs(np.asarray(Fm) - o.stage("Fmac")), axis=0) / tm))
    say(f"nv {len(c['u'])}: F {eF:.2e} Fmac {eFm:.2e} (against the face terms)")
    assert eF < 1e-6 and eFm < 1e-6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_unaligned_rows_take_the_scalar_kernels(precision):
    """Distribution and face arrays that start one element past an aligned address (the ABI requires element
    alignment only): the library then runs the scalar micro residual and micro sweep and the face kernel
    without LDS-DMA.  On the small sphere (1 944 tets x 1 288 velocities, which an aligned state runs through
    the 16-byte vector kernels and LDS-DMA), three iterations from rest give the aligned state's fields: the two
    paths do the same arithmetic per velocity (FP64 within 1e-12, FP32 rounding within 1e-6)."""
    from paper_2303_10846_amd.binding import Solver
    c = configs.small_sphere_case()
    say("case small_sphere", precision, "aligned and unaligned rows")
    states = []
    for off in (0, 1):
        s = Solver(c, precision=precision, row_offset=off)
        assert (s.G.data_ptr() % 16 == 0) == (off == 0)
        s.init_equilibrium(c["W0"])
        s.iterate(3)
        states.append(s.get_state())
        del s
    (Ga, Ra, Wa, qa), (Gu, Ru, Wu, qu) = states
    tol = 1e-12 if precision == "fp64" else 1e-6
    e = (nrel(Gu, Ga), nrel(Ru, Ra), colrel(Wu, Wa))
    say("unaligned against aligned: G %.2e R %.2e W %.2e" % e)
    assert max(e) < tol


def _grid_dvs(nx, ny, nz, half=4.0):
    """Midpoints of an nx x ny x nz grid on [-half, half]^3, weights the cell volumes."""
    ax = [(np.arange(n) + 0.5) * (2 * half / n) - half for n in (nx, ny, nz)]
    u = np.stack(np.meshgrid(*ax, indexing="ij"), -1).reshape(-1, 3)
    w = np.full(len(u), (2 * half) ** 3 / (nx * ny * nz))
    return u, w


def test_maximum_velocity_count():
    """nv = 16384, the library's limit, on the two-tet mesh: one iteration against the oracle (FP64); one more
    velocity is refused with CIS_E_UNSUPPORTED."""
    from paper_2303_10846_amd.binding import CisError
    u, w = _grid_dvs(32, 32, 16)
    c = dict(_tets_case(2), u=u, w=w)
    o, s = _pair(c, warm=1)
    o.iterate(1)
    s.iterate(1)
    G, R, W, q = s.get_state()
    Go, Ro, Wo, qo = o.get_state()
    assert nrel(G, Go) < TOL and nrel(R, Ro) < TOL and colrel(W, Wo) < TOL
    del s
    u1 = np.vstack([u, [[0.0, 0.0, 4.5]]])
    with pytest.raises(CisError) as e:
        solver(dict(c, u=u1, w=np.append(w, w[0])))
    assert e.value.status == -6


def test_converge_applies_the_step_schedule_and_stops_at_the_criterion():
    """Solver.converge: the implicit-step schedule takes effect at its iteration (the same history, bit for bit, as
    switching by hand), and the run stops at the first chunk whose residual is below the paper's 1e-10."""
    c = configs.cavity_case(n=2, nv_side=6)
    s1 = solver(c)
    s1.init_equilibrium(c["W0"])
    h1, ok = s1.converge(tol=1e-10, max_iter=600, cfl_schedule=[(0, 2.0), (40, 0.0)], chunk=50)
    say("converged after", len(h1), "iterations, residual", h1[-1].max())
    assert ok and h1[-1].max() < 1e-10 and len(h1) % 50 == 0 and len(h1) < 600
    if len(h1) > 50:
        assert np.all(h1[: len(h1) - 50].max(axis=1) >= 1e-10)  # not reached before the last chunk
    s2 = solver(c)
    s2.init_equilibrium(c["W0"])
    s2.set_numerics(cfl_imp=2.0)
    a = s2.iterate(40)
    s2.set_numerics(cfl_imp=0.0)
    b = s2.iterate(len(h1) - 40)
    assert np.array_equal(np.concatenate([a, b]), h1)
    # a run that stops at max_iter says so
    s3 = solver(c)
    s3.init_equilibrium(c["W0"])
    h3, ok3 = s3.converge(tol=1e-10, max_iter=20, chunk=10)
    assert not ok3 and len(h3) == 20 and h3[-1].max() >= 1e-10


def test_determinism_bitwise():
    c = configs.small_sphere_case()
    outs = []
    for _ in range(2):
        s = solver(c)
        s.init_equilibrium(c["W0"])
        s.iterate(3)
        outs.append(s.get_state())
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_uniform_free_stream_zero_residual_on_gpu():
    from paper_2303_10846_amd.cases import dvs
    U = np.array([0.3, -0.1, 0.2])
    c = configs.freestream_box_case(n=2, U=U, dvs=dvs.gauss_hermite_dvs(6, U, 1.0))
    s = solver(c)
    s.init_equilibrium(c["W0"])
    G0, _, W0, _ = s.get_state()
    h = s.iterate(2)
    G1, _, W1, _ = s.get_state()
    assert h.max() < 1e-14
    assert nrel(G1, G0) < 1e-13 and colrel(W1, W0) < 1e-14


def test_nonfinite_state_is_reported():
    """A negative density planted from the host is reported as CIS_E_NONFINITE (no kernel faults)."""
    from paper_2303_10846_amd.binding import CisError
    c = configs.cavity_case(n=2, nv_side=4)
    s = solver(c)
    s.init_equilibrium(c["W0"])
    G, R, W, q = s.get_state()
    W[3, 0] = -1.0
    s.set_state(G, R, W, q)
    with pytest.raises(CisError) as e:
        s.iterate(1)
    assert e.value.status == -5


def test_mixed_precision_cavity_converged_fields():
    """FP32 distributions and flux kernels, FP64 compensated moments/macro/diagonal: error of the
    converged density, temperature and wall heat flux against the FP64 oracle."""
    c = configs.cavity_case(seed=0)
    o = oracle.Oracle(c)
    o.init_equilibrium(c["W0"])
    o.iterate(200)
    _, _, Wo, _ = o.get_state()
    s = solver(c, precision="mixed")
    s.init_equilibrium(c["W0"])
    h = s.iterate(200)
    W, _ = s.moments()

    def rho_T(W):
        rho = W[:, 0]
        ke = 0.5 * np.sum(W[:, 1:4] ** 2, axis=1) / rho
        return rho, 0.4 * (W[:, 4] - ke) / (rho * 0.5)

    r, T = rho_T(W)
    ro, To = rho_T(Wo)
    er, eT = nrel(r, ro), nrel(T, To)
    eq = abs(s.wall_heat_flux(2) - o.wall_heat_flux(2)) / abs(o.wall_heat_flux(2))
    say(f"mixed vs FP64 oracle: rho {er:.2e} T {eT:.2e} Q_lid {eq:.2e}; final residual {h[-1].max():.2e}")
    assert er < 1e-5 and eT < 1e-5 and eq < 1e-5


@pytest.mark.parametrize("dims", [(8, 8, 4), (9, 9, 6), (7, 7, 7)])
def test_mixed_micro_sweep_vector_widths(dims):
    """The mixed micro sweep and micro residual move 4, 2 or 1 velocities per thread as one vector, by nv mod 4
    (256, 486, 343 velocities here): one mixed iteration from the oracle's state against the FP64 oracle's.  The bar is FP32
    rounding (6e-8) of phi amplified by the cancellation in Res = (phi* - phi)/tau - F, whose terms are up to
    ~1e3 times Res on this nearly resting cavity: measured 0.6-2.2e-5 for all three widths, and the same with
    the one-velocity kernel alone.  A wrong upstream value or upwind bit gives O(1) errors."""
    u, w = _grid_dvs(*dims)
    c = dict(configs.cavity_case(n=3, nv_side=4), u=u, w=w)
    say("case cavity n=3, nv", len(u))
    o = oracle.Oracle(c)
    o.init_equilibrium(c["W0"])
    o.iterate(3)
    G, R, W, q = o.get_state()
    s = solver(c, precision="mixed")
    s.set_state(G, R, W, q)
    o.iterate(1)
    s.iterate(1)
    eG = nrel(s.dG.cpu().numpy(), o.stage("dG"))
    eR = nrel(s.dR.cpu().numpy(), o.stage("dR"))
    Wm, _ = s.moments()
    eW = colrel(Wm, o.get_state()[2])
    say(f"mixed vs FP64 oracle: dG {eG:.2e} dR {eR:.2e} W {eW:.2e}")
    assert eG < 1e-4 and eR < 1e-4 and eW < 1e-4


def test_mixed_vector_kernels_on_the_small_sphere_stage_by_stage():
    """The mixed path's vector kernels (four velocities per thread: the small sphere's DVS has 1 288 points) against
    the FP64 oracle, stage by stage, on a state ten iterations from rest, where the flow is far from steady and Res
    is not dominated by cancellation.  Both sides start from the same FP32-rounded distributions, so every
    difference is FP32 arithmetic in the kernels.  Bars (normwise, against the largest oracle value of each array):
    the micro flux F and Res are sums of a few FP32 products whose terms are up to ~10x the result, so some tens
    of units of FP32 rounding (6e-8) of the largest term: measured F 6.6e-7, Fmac 7.1e-7, Res 1.4e-6; bar 4e-6
    (F) and 6e-6 (Res).  The increments inherit Res's error through an FP64 diagonal (measured 1.0e-6, bar 6e-6)
    and the updated moments are FP64 sums of them (measured 1.7e-7, bar 1e-6).  A wrong upwind bit, neighbour
    or equilibrium coefficient gives errors of order one."""
    say("case small_sphere mixed stage by stage")
    c = configs.small_sphere_case()
    assert len(c["u"]) % 4 == 0
    o = oracle.Oracle(c)
    o.init_equilibrium(c["W0"])
    o.iterate(10)
    G, R, W, q = o.get_state()
    G32, R32 = G.astype(np.float32), R.astype(np.float32)
    o.set_state(G32.astype(np.float64), R32.astype(np.float64), W, q)
    s = solver(c, precision="mixed")
    s.set_state(G32, R32, W, q)
    # explicit operator: micro flux (Eq. 31) and macro flux (Eq. 37)
    FG, FR, Fm = s.residual()
    o.explicit()
    eF = max(nrel(FG.cpu().numpy(), o.stage("FG")), nrel(FR.cpu().numpy(), o.stage("FR")))
    eFm = colrel(Fm, o.stage("Fmac"))
    # one iteration: Res (Eq. 33 right-hand side), the increments, the update
    s.set_state(G32, R32, W, q)
    s.iterate(1)
    o.iterate(1)
    eRes = max(nrel(s.resG.cpu().numpy(), o.stage("ResG")), nrel(s.resR.cpu().numpy(), o.stage("ResR")))
    ed = max(nrel(s.dG.cpu().numpy(), o.stage("dG")), nrel(s.dR.cpu().numpy(), o.stage("dR")))
    Wm, qm = s.moments()
    _, _, Wo, qo = o.get_state()
    eW = colrel(Wm, Wo)
    say(f"mixed vector kernels vs FP64 oracle: F {eF:.2e} Fmac {eFm:.2e} Res {eRes:.2e} dphi {ed:.2e} W {eW:.2e}")
    assert eF < 4e-6 and eFm < 4e-6 and eRes < 6e-6 and ed < 6e-6 and eW < 1e-6


def test_wall_loads_match_oracle_face_fluxes():
    """Per-face pressure, shear and heat flux (Eqs. 70-72 numerators) and the integrated force and heat load on
    the sphere wall, against the oracle's face macro fluxes on the same state."""
    say("case small_sphere wall loads")
    c = configs.small_sphere_case()
    o, s = _pair(c, warm=4)
    o.explicit()
    g = o.geometry()
    fm = o.stage("ffmac").reshape(-1, 6)
    n = g["n"].reshape(-1, 3)
    wall = (g["fn"] < 0) & (g["ftag"] == 1)
    A = g["A"][wall]
    mom = fm[wall, 1:4] / A[:, None]
    p = np.einsum("ij,ij->i", mom, n[wall])
    tau = mom - p[:, None] * n[wall]
    q = fm[wall, 4] / A
    L = s.wall_loads(1)
    assert len(L["p"]) == int(wall.sum())
    # the library and the oracle number faces independently: match them by centroid (nearest neighbour; the
    # two compute centroids in different summation orders, so equal coordinates may differ in the last bit)
    from scipy.spatial import cKDTree
    xo = g["xf"].reshape(-1, 3)[wall]
    dist, nearest = cKDTree(L["x"]).query(xo)
    assert np.max(dist) < 1e-12 and len(np.unique(nearest)) == len(nearest)
    oo, ol = np.arange(len(xo)), nearest
    p, tau, q = p[oo], tau[oo], q[oo]
    L = dict(L, x=L["x"][ol], area=L["area"][ol], n=L["n"][ol], p=L["p"][ol], tau=L["tau"][ol], q=L["q"][ol])
    assert nrel(L["p"], p) < TOL
    assert nrel(L["tau"], tau) < TOL
    assert nrel(L["q"], q) < TOL
    assert nrel(L["force"], fm[wall, 1:4].sum(axis=0)) < TOL
    assert abs(L["heat"] - fm[wall, 4].sum()) <= TOL * abs(fm[wall, 4].sum())
    assert abs(L["heat"] - s.wall_heat_flux(1)) <= 1e-14 * abs(L["heat"])
    from paper_2303_10846_amd.binding import wall_coefficients
    # the per-face loads integrate to the library's force
    f = L["area"][:, None] * (L["p"][:, None] * L["n"] + L["tau"])
    assert nrel(f.sum(axis=0), L["force"]) < 1e-12
    cf = wall_coefficients(L, 1.0, c["U_inf"], 1.0, A_ref=0.25 * np.pi)
    say(f"Cd {cf['Cd']:.4f}  Cl {cf['Cl']:.2e}  Cm {cf['Cm']:.2e}  CQ {cf['CQ']:.4f}  Cp max {cf['Cp'].max():.3f}")
    assert np.all(np.isfinite(cf["Cp"])) and cf["Cd"] > 0.0
    # a sphere at zero incidence: lift and pitching moment about its centre are small beside the drag
    assert abs(cf["Cl"]) < 0.05 * cf["Cd"] and abs(cf["Cm"]) < 0.05 * cf["Cd"]
    # cis_wall_coefficients on the state against the Eqs. 70-72 normalisation of the oracle's face fluxes
    U = np.asarray(c["U_inf"], dtype=float)
    Um = float(np.linalg.norm(U))
    qd = 0.5 * 1.0 * Um * Um
    A_ref, L_ref, x_ref = 0.25 * np.pi, 0.5, np.array([0.1, -0.2, 0.05])
    co = s.wall_coefficients(1, 1.0, U, 1.0, A_ref=A_ref, L_ref=L_ref, x_ref=x_ref, lift_dir=(0.0, 1.0, 0.0))
    assert nrel(co["Cp"][ol], (p - 1.0 * 0.5 * 1.0) / qd) < TOL
    assert nrel(co["Ctau"][ol], np.linalg.norm(tau, axis=1) / qd) < TOL
    assert nrel(co["Ch"][ol], q / (qd * Um)) < TOL
    Fo = fm[wall, 1:4].sum(axis=0)
    Mo = np.cross(g["xf"].reshape(-1, 3)[wall] - x_ref, fm[wall, 1:4]).sum(axis=0)
    eD, eL = U / Um, np.array([0.0, 1.0, 0.0])
    assert nrel(co["CF"], Fo / (qd * A_ref)) < TOL
    assert abs(co["Cd"] - Fo @ eD / (qd * A_ref)) <= TOL * abs(Fo @ eD / (qd * A_ref))
    assert abs(co["Cl"] - Fo @ eL / (qd * A_ref)) <= TOL * np.max(np.abs(Fo)) / (qd * A_ref)
    assert nrel(co["CM"], Mo / (qd * A_ref * L_ref)) < TOL
    assert abs(co["Cm"] - co["CM"] @ np.cross(eL, eD)) <= 1e-14 * np.max(np.abs(co["CM"]))
    assert abs(co["CQ"] - fm[wall, 4].sum() / (qd * Um * A_ref)) <= TOL * abs(co["CQ"])


def test_no_micro_sweeps_means_zero_increments():
    """n_micro = 0: Eq. 33 is not swept, the increments are zero and the update keeps phi^n (stage-by-stage)."""
    say("case cavity n_micro 0")
    c = configs.cavity_case(n=2, nv_side=4)
    num = dict(c["num"], n_micro=0)
    o, s = _pair(c, warm=2, num=num)
    o.iterate(1)
    s.iterate(1)
    Go, Ro, Wo, qo = o.get_state()
    Gs, Rs, Ws, qs = s.get_state()
    assert nrel(Gs, Go) < TOL and nrel(Rs, Ro) < TOL
    assert colrel(Ws, Wo) < TOL and colrel(qs, qo) < TOL


@pytest.mark.parametrize("name", ["cavity_n3_dvs7", "small_sphere"])
def test_upwind_codes_match_oracle_decisions(name):
    """The per-(cell, velocity) upwind codes written by cis_state_create: for face slot a (the face opposite local
    vertex a) 1 where u.n out of the cell exceeds the tie tolerance, 2 where it is below minus it, 0 otherwise,
    against the oracle's geometry; and the two cells of an interior face see opposite codes."""
    say("case", name, "upwind codes")
    c = CASES[name]()
    o = oracle.Oracle(c)
    g = o.geometry()
    s = solver(c)
    codes = s.upwind.cpu().numpy().astype(np.int64)
    u = np.asarray(c["u"], dtype=np.float64)
    snap = c["num"]["snap"] * np.linalg.norm(u, axis=1)
    nc = codes.shape[0]
    want = np.zeros_like(codes)
    for a in range(4):
        f = g["cf"][:, a]
        sign = np.where(g["fo"][f] == np.arange(nc), 1.0, -1.0)
        un = (u @ g["n"][f].T).T * sign[:, None]                      # [nc][nv]
        ca = np.where(un > snap[None, :], 1, np.where(un < -snap[None, :], 2, 0))
        want |= ca << (2 * a)
    assert np.array_equal(codes, want)
    # opposite codes across every interior face
    for a in range(4):
        f = g["cf"][:, a]
        j = np.where(g["fo"][f] == np.arange(nc), g["fn"][f], g["fo"][f])
        inner = j >= 0
        b = np.argmax(g["cf"][j[inner]] == f[inner, None], axis=1)
        ci = (codes[inner] >> (2 * a)) & 3
        cj = (codes[j[inner]] >> (2 * b[:, None])) & 3
        assert np.array_equal(np.where(ci == 0, 0, 3 - ci), cj)
