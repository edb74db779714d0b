"""Checks at the full sizes of the synthetic workloads, in the launch configuration bench.py times.

* sphere (50k tets x 4k velocities, FP64): one iteration from rest against the oracle at full size;
* capsule mesh (303k tets) with a coarse DVS from the same generator: mixed path against the FP64 oracle;
* full capsule configuration (303k tets x 10.6k velocities, 3.2e9 pairs, mixed): the result must not depend on
  the order of the discrete velocities (equivariance under a permutation of the DVS), a property that holds at
  any size and would expose offset errors above 2^31 elements;
* the Ma 10 capsule on its hexahedral O-grid with the full DVS: convergence to the paper's criterion, the adjoint
  gradient against central differences and the mixed fields against the FP64 ones, all at the converged state;
* the VJP of the steady residual at the sphere's full size, and at the capsule's mesh size with a coarse DVS,
  against central differences of the GPU steady residual along a random direction (state and parameters): <v, R(x + e u) - R(x - e u)>/2e + cJ (J+ - J-)/2e
  = <VJP(v, cJ), u>.  With the limiter off the residual is smooth and the two agree to 1e-9.  With it on, the
  limiter's switching points (min over faces, extremum neighbours) crossed by the perturbation make the
  difference quotient a poor reference (4e-3 measured at step 1e-8, falling only linearly with the step), so
  that check only guards against gross errors; the limiter branch of the VJP is checked exactly against the
  oracle's complex-step JVP, which follows the same branches, in test_gpu_adjoint.py.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2303_10846_amd.cases import configs

pytestmark = pytest.mark.gpu


def nrel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def colrel(a, b):
    return max(nrel(a[:, m], b[:, m]) for m in range(a.shape[1]))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_sphere_full_size_one_iteration_fp64():
    from paper_2303_10846_amd.binding import Solver
    c = configs.sphere_case(seed=0)
    say("case", c["name"], len(c["mesh"]["tets"]), "x", len(c["u"]))
    s = Solver(c, precision="fp64")
    s.init_equilibrium(c["W0"])
    hs = s.iterate(1)
    W, q = s.moments()
    dW = s.debug_stage("dW")
    Gs, _, _, _ = s.get_state()
    del s
    o = oracle.Oracle(c)
    o.init_equilibrium(c["W0"])
    ho = o.iterate(1)
    Go, _, Wo, qo = o.get_state()
    say(f"W {colrel(W, Wo):.2e} q {colrel(q, qo):.2e} dW {colrel(dW, o.stage('dW')):.2e} G {nrel(Gs, Go):.2e}")
    assert colrel(W, Wo) < 1e-11
    assert colrel(dW, o.stage("dW")) < 1e-11
    assert colrel(q, qo) < 1e-10
    assert nrel(Gs, Go) < 1e-11
    assert np.max(np.abs(hs - ho) / np.abs(ho)) < 1e-9


def test_sphere_full_size_one_iteration_mixed():
    """The headline path itself: the mixed precision on the full sphere workload (LDS-DMA face staging, vector
    micro kernels, 4 140 velocities), one iteration from rest against the FP64 oracle.  The GPU starts from its
    FP32 equilibrium, so both the initial state and the arithmetic differ by FP32 rounding (6e-8 of the largest
    terms): bars 2e-6 on W (normwise per quantity: rho, the momentum vector, rho E, rho E_rot) and 1e-4 on the
    wall heat load, a sum over incoming and outgoing velocities that cancels to a few per cent of its terms.  A
    wrong staged value, upwind bit or coefficient gives errors of order one."""
    from paper_2303_10846_amd.binding import Solver
    c = configs.sphere_case(seed=0)
    say("case", c["name"], "mixed", len(c["mesh"]["tets"]), "x", len(c["u"]))
    s = Solver(c, precision="mixed")
    s.init_equilibrium(c["W0"])
    s.iterate(1)
    W, _ = s.moments()
    Qw = s.wall_heat_flux(1)
    del s
    o = oracle.Oracle(c)
    o.init_equilibrium(c["W0"])
    o.iterate(1)
    _, _, Wo, _ = o.get_state()
    Qo = o.wall_heat_flux(1)
    mom = float(np.max(np.abs(Wo[:, 1:4])))
    scale = np.array([np.max(np.abs(Wo[:, 0])), mom, mom, mom, np.max(np.abs(Wo[:, 4])), np.max(np.abs(Wo[:, 5]))])
    eW = float(np.max(np.max(np.abs(W - Wo), axis=0) / scale))
    eQ = abs(Qw - Qo) / abs(Qo)
    say(f"mixed full sphere vs oracle: W {eW:.2e} Q_w {eQ:.2e}")
    assert eW < 2e-6 and eQ < 1e-4


def test_capsule_mesh_full_size_coarse_dvs_mixed_vs_oracle():
    from paper_2303_10846_amd.binding import Solver
    c = configs.capsule_case(seed=0, nv_target=700)
    say("case", c["name"], len(c["mesh"]["tets"]), "x", len(c["u"]))
    s = Solver(c, precision="mixed")
    s.init_equilibrium(c["W0"])
    s.iterate(2)
    W, q = s.moments()
    del s
    o = oracle.Oracle(c)
    o.init_equilibrium(c["W0"])
    o.iterate(2)
    _, _, Wo, _ = o.get_state()
    e = colrel(W, Wo)
    say(f"mixed vs FP64 oracle after 2 iterations: W {e:.2e}")
    assert e < 1e-5


def test_capsule_full_config_mixed_dvs_permutation_equivariance():
    import torch

    from paper_2303_10846_amd.binding import Solver
    c = configs.capsule_case(seed=0)
    pairs = len(c["mesh"]["tets"]) * len(c["u"])
    say("case", c["name"], len(c["mesh"]["tets"]), "x", len(c["u"]), f"pairs {pairs:.3g}")
    assert pairs > 2 ** 31
    res = []
    perm = np.random.default_rng(5).permutation(len(c["u"]))
    for cc in (c, dict(c, u=c["u"][perm], w=c["w"][perm])):
        s = Solver(cc, precision="mixed")
        s.init_equilibrium(cc["W0"])
        h = s.iterate(2)
        W, q = s.moments()
        Q = s.wall_heat_flux(1)
        say(f"  residual {h[-1].max():.3e} Q_w {Q:.6e}")
        assert np.all(np.isfinite(h)) and np.all(np.isfinite(W))
        res.append((W, q, Q))
        del s
        torch.cuda.empty_cache()
    (W1, q1, Q1), (W2, q2, Q2) = res
    say(f"W {colrel(W2, W1):.2e} q {colrel(q2, q1):.2e} Q {abs(Q2 - Q1) / abs(Q1):.2e}")
    # the same velocities in another order: equal up to FP32 summation-order rounding
    assert colrel(W2, W1) < 1e-5
    assert abs(Q2 - Q1) < 1e-5 * abs(Q1)


def _sphere_vjp_fd(limiter, eps, tol, case=None, warm=20):
    import torch
    from paper_2303_10846_amd.binding import Solver
    c = case if case is not None else configs.sphere_case(seed=0)
    s = Solver(c, precision="fp64")
    s.init_equilibrium(c["W0"])
    s.iterate(warm)                     # a developed, non-steady state (limiter on, as the case runs)
    if limiter == 3:
        s.freeze_limiter()              # the limiter values of this state, held fixed: a smooth residual
    else:
        s.set_numerics(limiter=limiter)
    gen = torch.Generator(device=s.device).manual_seed(7)
    rnd = lambda t: torch.randn(t.shape, generator=gen, device=s.device, dtype=t.dtype)  # noqa: E731
    v = [rnd(s.G), rnd(s.R), rnd(s.W), rnd(s.q)]
    u = [rnd(s.G) * s.G.abs(), rnd(s.R) * s.R.abs(), rnd(s.W) * 1e-3, rnd(s.q) * 1e-4]
    up = np.array([0.3, 0.2, 0.1])
    cJ = 0.5
    gG, gR, gW, gq, gp = s.residual_vjp(*v, cJ=cJ, wall_tag=1, ff_tag=2)
    rhs = sum(float((g * du).sum()) for g, du in zip((gG, gR, gW, gq), u)) + float(gp @ up)
    del gG, gR, gW, gq
    x0 = [t.clone() for t in (s.G, s.R, s.W, s.q)]
    p0 = s.params(1, 2)
    out = []
    for sg in (1, -1):
        for t, b, du in zip((s.G, s.R, s.W, s.q), x0, u):
            t.copy_(b + sg * eps * du)
        s.set_params(p0 + sg * eps * up, 1, 2)
        rG, rR, rW, rq, J = s.steady_residual(1)
        out.append((sum(float((vv * r).sum()) for vv, r in zip(v, (rG, rR, rW, rq))), J))
        del rG, rR, rW, rq
    lhs = (out[0][0] - out[1][0]) / (2 * eps) + cJ * (out[0][1] - out[1][1]) / (2 * eps)
    say(f"limiter {limiter}: lhs {lhs:.12e} rhs {rhs:.12e} rel {abs(lhs - rhs) / abs(rhs):.3e}")
    assert abs(lhs - rhs) <= tol * abs(rhs)


def test_sphere_full_size_vjp_smooth_residual():
    _sphere_vjp_fd(limiter=0, eps=1e-6, tol=1e-8)


def test_capsule_mesh_full_size_vjp_smooth_residual():
    """The VJP at the capsule's mesh size (303 264 tets, the Ma 10 capsule's gas and boundaries) in FP64, with the
    DVS coarsened to ~700 points so that the FP64 state, the seed, the perturbation and the gradient fit one GPU
    (the full 10 568-point DVS in FP64 would need ~26 GB per array, over 250 GB for the check); against central
    differences of the steady residual along a random direction.  The limiter values of the state are stored and
    held fixed (limiter 3), which keeps the residual smooth: with the limiter off, the unlimited reconstruction at
    the forming Ma 10 bow shock gives face states with negative temperature (NaN viscosity)."""
    c = configs.capsule_case(seed=0, nv_target=700)
    say("case", c["name"], len(c["mesh"]["tets"]), "x", len(c["u"]))
    _sphere_vjp_fd(limiter=3, eps=1e-6, tol=1e-8, case=c, warm=5)


def test_sphere_full_size_vjp_limited_residual():
    _sphere_vjp_fd(limiter=1, eps=1e-8, tol=2e-2)


def test_hexahedral_sphere_converges_to_the_paper_criterion():
    """The sphere workload's O-grid kept as hexahedra (the paper's sphere mesh is hexahedral, Sec. 4.2): 48 384
    cells x 4 140 velocities, FP64, from rest.  The residual falls below the paper's steady criterion (global
    average residual below 1e-10, Sec. 4.1) within 600 iterations, and Solver.converge goes on to 1e-12, where
    the heat load is steady to 10 digits over the last 100 iterations; the wall coefficients are those of a blunt
    body at zero incidence."""
    import math
    c = configs.sphere_hex_case(seed=0)
    say("case", c["name"], len(c["mesh"]["cells"]), "hexahedra x", len(c["u"]))
    from paper_2303_10846_amd.binding import Solver
    s = Solver(c, precision="fp64")
    s.init_equilibrium(c["W0"])
    qs = []
    h, ok = s.converge(tol=1e-12, max_iter=900, chunk=100, callback=lambda it, hh: qs.append(s.wall_heat_flux(1)))
    r = h.max(axis=1)
    first = int(np.argmax(r < 1e-10)) + 1
    say("converged", ok, "after", len(h), "iterations, residual", r[-1], "below 1e-10 at", first, "Q_w", qs[-3:])
    assert ok and r[-1] < 1e-12 and first <= 600
    assert abs(qs[-1] - qs[-2]) <= 1e-10 * abs(qs[-1])
    co = s.wall_coefficients(1, 1.0, c["U_inf"], 1.0, A_ref=0.25 * math.pi)
    say(f"Cd {co['Cd']:.5f} Cl {co['Cl']:.2e} CQ {co['CQ']:.5f}")
    assert 1.0 < co["Cd"] < 2.0 and abs(co["Cl"]) < 1e-3 * co["Cd"] and co["CQ"] > 0


@pytest.mark.timeout(600)
def test_hexahedral_capsule_converges_adjoint_and_mixed_precision():
    """The Ma 10 capsule on the hexahedral O-grid that the tetrahedral capsule splits (25 272 hexahedra x 10 568
    velocities, the full DVS; the paper's blunted-cone mesh is hexahedral, Sec. 4.3), from rest with the capsule's
    implicit-step schedule:

    * FP64 falls below the paper's criterion of 1e-10 (Sec. 4.1) within 1 400 iterations (measured 1 232) and
      goes on to 1e-13;
    * the adjoint gradient of the wall heat load with the limiter values stored at that state (limiter 3; GMRES(40)
      to 1e-10, 65 iterations) against central differences of the converged heat load with step 1e-6 of T_w:
      within 1e-6 (measured 1.5e-8);
    * mixed precision from rest to its rounding floor (~1.5e-6): density, temperature and heat load against the
      converged FP64 fields within 1e-5 (measured 1.4e-7, 9e-8, 2.6e-8);
    * the adjoint taken at the mixed-precision converged state (its FP32 distributions widened into the FP64
      state, limiter values stored there): dQ_w/dT_w within 1e-5 of the FP64 state's (measured 4.1e-6: the
      limiter values stored at the two states differ more than the fields)."""
    import math

    import bench
    c = configs.capsule_hex_case(seed=0)
    say("case", c["name"], len(c["mesh"]["cells"]), "hexahedra x", len(c["u"]))
    from paper_2303_10846_amd.binding import Solver
    s = Solver(c, precision="fp64")
    s.init_equilibrium(c["W0"])
    h, ok = s.converge(tol=1e-13, max_iter=2000, chunk=100, cfl_schedule=bench.CAPSULE_CFL_RAMP)
    r = h.max(axis=1)
    first = int(np.argmax(r < 1e-10)) + 1
    say("fp64 converged", ok, "after", len(h), "iterations, residual", r[-1], "below 1e-10 at", first)
    assert ok and first <= 1400
    co = s.wall_coefficients(1, 1.0, c["U_inf"], 1.0, A_ref=0.25 * math.pi)
    say(f"Cd {co['Cd']:.7f} Cl {co['Cl']:.2e} CQ {co['CQ']:.7f}")
    assert 1.0 < co["Cd"] < 2.0 and abs(co["Cl"]) < 1e-3 * co["Cd"] and co["CQ"] > 0
    W64, _ = s.moments()
    Q64 = s.wall_heat_flux(1)
    base = s.get_state()
    s.freeze_limiter()
    a = s.adjoint(1, 2, restart=40, max_iter=300, rtol=1e-10, precond_pairs=2, macro_pairs=20)
    say("stored-limiter adjoint", a["iterations"], "iterations, relative residual", a["rel_residual"],
        "dJ/dp", a["dJdp"])
    assert a["converged"]
    dJ = float(a["dJdp"][0])
    del a
    p0 = s.params(1, 2)
    hk = 1e-6 * abs(p0[0])
    J = []
    for sgn in (1, -1):
        p = p0.copy()
        p[0] += sgn * hk
        s.set_params(p, 1, 2)
        s.set_state(*base)
        hh, okk = s.converge(tol=1e-13, max_iter=600, chunk=50)
        assert okk
        J.append(s.wall_heat_flux(1))
    fd = (J[0] - J[1]) / (2 * hk)
    say(f"dQ_w/dT_w adjoint {dJ:.10f} central differences {fd:.10f}")
    assert abs(dJ - fd) <= 1e-6 * abs(fd)
    s.set_params(p0, 1, 2)
    s.unfreeze_limiter()
    del base
    m = Solver(c, precision="mixed")
    m.init_equilibrium(c["W0"])
    hm, _ = m.converge(tol=1e-10, max_iter=1300, chunk=100, cfl_schedule=bench.CAPSULE_CFL_RAMP)
    say("mixed after", len(hm), "iterations, residual", hm[-1].max())
    Wm, _ = m.moments()

    def rho_T(W):
        rho = W[:, 0]
        return rho, 0.4 * (W[:, 4] - 0.5 * np.sum(W[:, 1:4] ** 2, axis=1) / rho) / (0.5 * rho)

    (rm, Tm), (rd, Td) = rho_T(Wm), rho_T(W64)
    e = (nrel(rm, rd), nrel(Tm, Td), abs(m.wall_heat_flux(1) - Q64) / abs(Q64))
    say("mixed against fp64: rho %.2e T %.2e Q_w %.2e" % e)
    assert max(e) <= 1e-5
    Gm, Rm, Wm2, qm = m.get_state()
    del m
    s.set_state(Gm.astype(np.float64), Rm.astype(np.float64), Wm2, qm)
    s.freeze_limiter()
    am = s.adjoint(1, 2, restart=40, max_iter=300, rtol=1e-10, precond_pairs=2, macro_pairs=20)
    assert am["converged"]
    dJm = float(am["dJdp"][0])
    say(f"dQ_w/dT_w at the mixed state {dJm:.10f}, at the FP64 state {dJ:.10f}, relative {abs(dJm - dJ) / abs(dJ):.2e}")
    assert abs(dJm - dJ) <= 1e-5 * abs(dJ)


def test_hexahedral_sphere_adjoint_matches_central_differences():
    """The adjoint gradient of the sphere's wall heat load: the hexahedral sphere converged to a residual below
    1e-13 (FP64), dQ_w/dp for p = (T_w, rho_inf, |U_inf|) from the discrete adjoint (limiter differentiated on its
    branch, GMRES to 1e-10) against central differences of the converged heat load with step 1e-6 of each
    parameter: within 1e-6 (measured 1e-8 to 8e-8)."""
    c = configs.sphere_hex_case(seed=0)
    say("case", c["name"], "adjoint against central differences")
    from paper_2303_10846_amd.binding import Solver
    s = Solver(c, precision="fp64")
    s.init_equilibrium(c["W0"])
    h, ok = s.converge(tol=1e-13, max_iter=900, chunk=100)
    assert ok
    base = s.get_state()
    a = s.adjoint(1, 2, restart=60, max_iter=400, rtol=1e-10, precond_pairs=2, macro_pairs=20)
    say("adjoint", a["iterations"], "iterations, relative residual", a["rel_residual"], "dJ/dp", a["dJdp"])
    assert a["converged"]
    p0 = s.params(1, 2)
    for k in range(3):
        hk = 1e-6 * abs(p0[k])
        J = []
        for sgn in (1, -1):
            p = p0.copy()
            p[k] += sgn * hk
            s.set_params(p, 1, 2)
            s.set_state(*base)
            hh, okk = s.converge(tol=1e-13, max_iter=600, chunk=50)
            assert okk
            J.append(s.wall_heat_flux(1))
        fd = (J[0] - J[1]) / (2 * hk)
        say(f"p[{k}] adjoint {a['dJdp'][k]:.10f} central differences {fd:.10f}")
        assert abs(a["dJdp"][k] - fd) <= 1e-6 * abs(fd)
    s.set_params(p0, 1, 2)
