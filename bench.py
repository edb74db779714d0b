"""Throughput of one implicit iteration (Steps 2-6) on one MI355X.

Workload: Ma 5 flow over a sphere (Kn 0.1, Tw/T_inf = 3) on a 50 400-tet graded mesh with a 4 140-point
unstructured DVS, started from rest.  Metric: cell-velocity updates per second per implicit iteration, for the
mixed-precision path (FP32 distributions and flux kernels, FP64 moments, macro system, implicit diagonal and
update) and the FP64 path.  Inputs are generated on the host and copied to HBM before the timed region; the
timed region is K iterations on the GPU.  Both runs then continue to the converged plateau, where the mixed
fields are compared with the FP64 ones ("at matched error").

--workload capsule times the Ma 10 capsule instead (303 264 tets x 10 568 velocities, 3.2e9 pairs, about 156 GB
of mixed-precision state), mixed precision only.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def sweep_cells(color_offsets, n_pairs):
    """Cell relaxations of n_pairs forward + backward colour passes; a colour that follows itself at a turn
    of direction is relaxed once (the library skips the bitwise-identical repeat)."""
    off = np.asarray(color_offsets)
    seq = []
    for _ in range(n_pairs):
        for c in list(range(len(off) - 1)) + list(range(len(off) - 2, -1, -1)):
            if off[c + 1] > off[c] and (not seq or seq[-1] != c):
                seq.append(c)
    return int(sum(off[c + 1] - off[c] for c in seq))


def stage_bytes(nc, nf, nv, es, micro_cells):
    """Algorithmic HBM bytes of one iteration per stage (each value moved once)."""
    return {
        "recon": (2 * nc + 2 * nf) * nv * es,          # read phi (G, R); write phi_bar for every (face, velocity)
        "face": 4 * nf * nv * es,                      # read phi_bar; write A (u.n) phi_f
        "residual": (2 * nf + 4 * nc) * nv * es,       # read face fluxes and phi; write Res
        "micro": 6 * micro_cells * nv * es,            # per relaxation: read Res, neighbour dphi; write dphi
        "update": 6 * nc * nv * es,                    # read phi, dphi; write phi
    }


# Algorithmic words per (cell, velocity) of the scope table's byte model (one word = one G or R value):
# the face pass reads phi^n and writes the micro flux F (2 + 2), the residual reads phi^n and F and writes Res
# (6), each micro relaxation reads Res and the upstream increment and writes the increment (6 per relaxed cell),
# the update reads phi and dphi and writes phi (6).  Four half-sweeps give the model's 40 words per iteration.
MODEL_WORDS = {"face": 4, "residual": 6, "micro_per_relaxation": 6, "update": 6}
MODEL_WORDS_PER_ITER = 40


def model_bytes(nc, nv, es, micro_cells):
    """Algorithmic bytes per iteration of each stage by the scope table's per-(cell, velocity) words.  The
    face pass (reconstruction + face kernels) is charged to the face kernel, which it is timed against."""
    return {
        "face": MODEL_WORDS["face"] * nc * nv * es,
        "residual": MODEL_WORDS["residual"] * nc * nv * es,
        "micro": MODEL_WORDS["micro_per_relaxation"] * micro_cells * nv * es,
        "update": MODEL_WORDS["update"] * nc * nv * es,
    }


STAGE_KERNEL = {"recon": "k_recon", "face": "k_face", "residual": "k_residual", "micro": "k_micro_sweep",
                "update": "k_update"}


def roofline(stage, precision, alg_bytes_iter, ms_iter, launches_iter, workload="sphere", kernel_bytes_iter=None):
    """Roofline of one stage: algorithmic bytes per launch (the scope table's per-(cell, velocity) words, as
    alg_bytes_iter) over the average launch duration (hipEvents on the library's stream), and the
    counter-measured HBM bytes per launch when the committed rocprofv3 summary still matches the kernel sources.
    kernel_bytes_iter, if given, is the same stage under the per-kernel model (every value the kernel itself
    reads or writes, once), reported beside it as `kernel_model`."""
    from paper_2303_10846_amd import prof_summary
    per_launch = alg_bytes_iter / launches_iter
    t_launch = ms_iter * 1e-3 / launches_iter
    ach = per_launch / t_launch / 1e9
    out = {"kernel": STAGE_KERNEL[stage], "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": ach / HBM_PEAK_GBS, "traffic": None, "launches_per_iter": launches_iter,
           "algorithmic_bytes_per_launch": per_launch, "avg_launch_us": t_launch * 1e6,
           "byte_model": "scope table words per (cell, velocity)"}
    if kernel_bytes_iter is not None:
        kb = kernel_bytes_iter / launches_iter
        out["kernel_model"] = {"bytes_per_launch": kb, "achieved": kb / t_launch / 1e9,
                               "frac": kb / t_launch / 1e9 / HBM_PEAK_GBS,
                               "basis": "every value the kernel reads or writes, once"}
    path = os.path.join(ROOT, "profiles", f"{stage}_{precision}_{workload}_counters.txt")
    if os.path.exists(path):
        c = prof_summary.read_counters(path)
        if c.get("source_sha256") == prof_summary.source_hash() and STAGE_KERNEL[stage] in c.get("kernel", ""):
            tb = float(c["hbm_bytes_per_dispatch"])
            out["kernel"] = c["kernel"]
            out["traffic"] = tb
            out["traffic_GBs"] = tb / t_launch / 1e9
            out["traffic_frac"] = tb / t_launch / 1e9 / HBM_PEAK_GBS
            out["traffic_over_algorithmic"] = tb / per_launch
            out["traffic_source"] = os.path.relpath(path, ROOT)
    # VALU issue time of the same kernel (SQ_INSTS_VALU, 4 cycles per wavefront instruction) as a fraction of
    # its duration: how close the kernel is to the instruction-issue bound
    sq_path = os.path.join(ROOT, "profiles", f"sq_{precision}_{workload}_counters.txt")
    if os.path.exists(sq_path):
        lines = open(sq_path).read().splitlines()
        if any(l.strip() == f"# source_sha256: {prof_summary.source_hash()}" for l in lines[:4]):
            cur = None
            for l in lines:
                if l.startswith("kernel:"):
                    cur = l.split(":", 1)[1].strip()
                elif cur and STAGE_KERNEL[stage] in cur and l.strip().startswith("valu_issue_us:"):
                    out["valu_issue_frac"] = float(l.split(":", 1)[1]) / (t_launch * 1e6)
                    out["valu_source"] = os.path.relpath(sq_path, ROOT)
                    break
    return out


def run_path(case, precision, steps, warmup, converge_iters, workload="sphere"):
    import torch

    from paper_2303_10846_amd.binding import Solver
    s = Solver(case, precision=precision, device="cuda:0")
    s.init_equilibrium(case["W0"])
    hists = []
    if warmup:
        hists.append(s.iterate(warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = s.iterate(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    hists.append(hist)
    # stage times with hipEvents on the solver's stream, over a second timed region of the same length
    s.profile(True)
    hists.append(s.iterate(steps))
    prof = s.profile_read()
    s.profile(False)
    # continue to the converged plateau for the comparison of the two precisions (not timed)
    done = warmup + 2 * steps
    while done < converge_iters:
        n = min(200, converge_iters - done)
        hist = s.iterate(n)
        hists.append(hist)
        done += n
        print(f"bench: {precision} {done} iterations, residual {hist[-1].max():.3e}", file=sys.stderr, flush=True)
    W, q = s.moments()
    Qw = s.wall_heat_flux(1)
    # iterations from rest until the residual (max over the six components) first falls below each level
    res = np.concatenate(hists).max(axis=1)
    to_level = {f"{lv:.0e}": (int(np.argmax(res <= lv)) + 1 if np.any(res <= lv) else None) for lv in (1e-4, 1e-5, 1e-6)}
    pairs = s.nc * s.nv
    es = 8 if precision == "fp64" else 4
    mcells = sweep_cells(case["mesh"]["color_offsets"], case["num"]["n_micro"])
    sb = stage_bytes(s.nc, s.nf, s.nv, es, mcells)
    mb = model_bytes(s.nc, s.nv, es, mcells)
    stages = {}
    for k, (ms, nl) in prof.items():
        e = dict(ms_per_iter=ms / steps, launches_per_iter=nl / steps)
        if k in sb:
            e["kernel_GB_per_iter"] = sb[k] / 1e9
            e["kernel_GBs"] = sb[k] * steps / (ms * 1e-3) / 1e9 if ms > 0 else None
        if k in mb:
            e["algorithmic_GB_per_iter"] = mb[k] / 1e9
            e["achieved_GBs"] = mb[k] * steps / (ms * 1e-3) / 1e9 if ms > 0 else None
        stages[k] = e
    hbm = {k: v for k, v in stages.items() if k in mb}
    dom = max(hbm, key=lambda k: hbm[k]["ms_per_iter"])
    roof = roofline(dom, precision, mb[dom], prof[dom][0] / steps, prof[dom][1] / steps, workload, sb[dom])
    # the micro sweep (the HBM-bound implicit sweep) beside the dominant kernel when that is another one
    roof_sweep = (roofline("micro", precision, mb["micro"], prof["micro"][0] / steps, prof["micro"][1] / steps,
                           workload, sb["micro"]) if dom != "micro" and "micro" in prof and prof["micro"][1]
                  else None)
    # the whole iteration against the scope table's 40 words per (cell, velocity)
    t_iter = t / steps
    it_bytes = MODEL_WORDS_PER_ITER * pairs * es
    roof_iter = {"bound": "hbm", "achieved": it_bytes / t_iter / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": it_bytes / t_iter / 1e9 / HBM_PEAK_GBS, "bytes_per_iteration": it_bytes,
                 "words_per_pair": MODEL_WORDS_PER_ITER, "ms_per_iteration": 1e3 * t_iter}
    out = dict(value=pairs * steps / t, ms_per_step=1e3 * t / steps, pairs=pairs, n_cells=s.nc, n_faces=s.nf,
               n_vel=s.nv, residual_last=float(hist[-1].max()), iterations=max(done, warmup + 2 * steps),
               stages=stages, roofline=roof, roofline_sweep=roof_sweep, roofline_iteration=roof_iter, Qw=Qw, W=W,
               iterations_to=to_level)
    del s
    torch.cuda.empty_cache()
    return out


def _oracle_rate(case, stride, iters):
    """Cell-velocity updates/s of the oracle on `case` with every `stride`-th velocity (the median over `iters`
    separately timed iterations), and the seconds taken in all."""
    import oracle
    c = dict(case, u=case["u"][::stride], w=case["w"][::stride] * stride) if stride > 1 else case
    o = oracle.Oracle(c)
    o.init_equilibrium(c["W0"])
    ts = []
    for _ in range(iters):
        t0 = time.perf_counter()
        o.iterate(1)
        ts.append(time.perf_counter() - t0)
    return o.nc * o.nv / float(np.median(ts)), float(sum(ts)), o.nc, o.nv


def cpu_baseline(case, stride=1, iters=3, stride_1t=32, iters_1t=2):
    """The oracle on the whole sphere workload (every velocity; `stride` > 1 samples the DVS), the median of
    `iters` iterations from rest, on all host threads; then on one thread with every `stride_1t`-th velocity."""
    import oracle
    cores = oracle.threads()
    value, t, nc, nv = _oracle_rate(case, stride, iters)
    oracle.threads(1)
    try:
        value_1t, t_1t, _, nv_1t = _oracle_rate(case, stride_1t, iters_1t)
    finally:
        oracle.threads(cores)
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            model = next(line.split(":", 1)[1].strip() for line in f if line.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": value, "unit": "cell-velocity updates/s", "cores": cores, "kind": "oracle",
            "sample": (f"the sphere workload ({nc} tets x all {nv} velocities)" if stride == 1 else
                       f"sphere mesh {nc} tets x one DVS point in {stride} ({nv} of {len(case['u'])})") +
                      f", median of {iters} FP64 iterations from rest ({t:.1f} s in all), {cores} OpenMP threads "
                      f"on {model}",
            "paper_context": "the paper's implicit solver: about 7.0e7-8.4e7 pairs/s with MPI over the DVS on "
                             "240-280 Xeon 6248R cores, derived from its timing tables (Tables 1 and 3) and mesh "
                             "sizes, and a speedup of 14-194x in wall time to convergence over the explicit "
                             "conserved DUGKS on the same cores; other hardware and meshes, not a target",
            "single_thread": {"value": value_1t, "cores": 1,
                              "sample": f"one DVS point in {stride_1t} ({nv_1t}), median of {iters_1t} "
                                        f"iterations ({t_1t:.1f} s)"}}


# DVS sets of the velocity-space study on the sphere: (name, outer radius / sqrt(R T0), target count).  Like the
# paper's capsule series (Sec. 4.4, Table 7), the first four shrink the spacing inside a ball of radius
# 5 sqrt(R T0) and the last two shrink the ball to 4 and 3 sqrt(R T0); every set keeps the refined balls of
# Eq. 74 at the free-stream and wall velocities.
DVS_STUDY = (("V1", 5.0, 16000), ("V2", 5.0, 12000), ("V3", 5.0, 8000), ("V4", 5.0, 4096), ("V5", 4.0, 3000),
             ("V6", 3.0, 2000))
# On the capsule: the timed workload's set (10 568 velocities in the 5 sqrt(R T0) ball), a coarser spacing and
# the two smaller balls.
CAPSULE_DVS_STUDY = (("C2", 5.0, 6000), ("C3", 4.0, 4500), ("C4", 3.0, 3500))


def _coefficients(s, case, T_inf=1.0, gas_R=0.5):
    from paper_2303_10846_amd.binding import wall_coefficients
    co = wall_coefficients(s.wall_loads(1), 1.0, case["U_inf"], T_inf, gas_R, A_ref=math.pi * 0.25)
    return dict(Cd=co["Cd"], CQ=float(co["CQ"]), Cp_max=float(co["Cp"].max()), Ch_max=float(co["Ch"].max()))


def dvs_study(iters, workload="sphere"):
    """Aerodynamic coefficients of the Ma 5 sphere against the size and extent of the DVS (mixed precision,
    `iters` iterations from rest each), with relative differences against the finest set."""
    if workload == "capsule":
        return capsule_dvs_study(iters)
    import torch

    from paper_2303_10846_amd.binding import Solver, wall_coefficients
    from paper_2303_10846_amd.cases import configs, dvs
    case = configs.sphere_case(seed=0)
    gas_R, T_inf, tw, mach = 0.5, 1.0, case["T_w"], case["mach"]
    T0 = dvs.total_temperature(T_inf, mach)
    rows = []
    for name, factor, target in DVS_STUDY:
        u, w = dvs.paper_unstructured_dvs(case["U_inf"], T_inf, tw, mach, factor, target=target)
        c = dict(case, u=u, w=w)
        print(f"bench: dvs study {name}: radius {factor} sqrt(R T0), {len(u)} velocities", file=sys.stderr,
              flush=True)
        s = Solver(c, precision="mixed", device="cuda:0")
        s.init_equilibrium(c["W0"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, hist = 0, None
        while done < iters:
            n = min(200, iters - done)
            hist = s.iterate(n)
            done += n
            print(f"bench: dvs study {name} {done} iterations, residual {hist[-1].max():.3e}", file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        co = wall_coefficients(s.wall_loads(1), 1.0, case["U_inf"], T_inf, gas_R, A_ref=math.pi * 0.25)
        rows.append(dict(name=name, radius_over_sqrt_RT0=factor,
                         radius=factor * math.sqrt(gas_R * max(T0, tw)), n_vel=len(u),
                         ball_volume_covered=float(w.sum() / (4.0 / 3.0 * math.pi *
                                                              (factor * math.sqrt(gas_R * max(T0, tw))) ** 3)),
                         Cd=co["Cd"], CQ=float(co["CQ"]), Cp_max=float(co["Cp"].max()), Ch_max=float(co["Ch"].max()),
                         residual=float(hist[-1].max()), ms_per_iter=1e3 * t / iters))
        del s
        torch.cuda.empty_cache()
    ref = rows[0]
    for r in rows:
        r["rel_diff_vs_" + ref["name"]] = {k: (r[k] - ref[k]) / abs(ref[k]) for k in ("Cd", "CQ", "Cp_max", "Ch_max")}
    return {"study": "DVS size and extent, sphere Ma 5 Kn 0.1 Tw/Tinf 3", "n_cells": len(case["mesh"]["tets"]),
            "iterations": iters, "precision": "mixed", "A_ref": "pi d^2 / 4", "sets": rows}


def adjoint_check(gmres_iters=300, fd_rel=1e-3, fd_iters=400):
    """Discrete adjoint of the FP64 sphere at its converged plateau against central differences of the
    converged heat load.  The limiter is held fixed in the adjoint (limiter = 2, block preconditioner); the
    adjoint with the limiter differentiated on its active branch (limiter = 1) is run beside it for 60 GMRES
    iterations to show where it stands."""
    import torch

    from paper_2303_10846_amd.binding import Solver
    from paper_2303_10846_amd.cases import configs
    case = configs.sphere_case(seed=0)
    case["num"] = dict(case["num"], limiter=2)
    s = Solver(case, precision="fp64", device="cuda:0")
    s.init_equilibrium(case["W0"])
    hist = s.iterate(600)
    print(f"bench: adjoint check primal residual {hist[-1].max():.3e}", file=sys.stderr, flush=True)
    base = s.get_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a = s.adjoint(1, 2, restart=50, max_iter=gmres_iters, rtol=1e-8, precond_pairs=2, macro_pairs=20)
    t_adj = time.perf_counter() - t0
    print(f"bench: frozen-limiter adjoint {a['iterations']} iterations, relative residual {a['rel_residual']:.2e}",
          file=sys.stderr, flush=True)
    del a["lam"]
    torch.cuda.empty_cache()
    s.set_numerics(limiter=1)
    act = s.adjoint(1, 2, restart=20, max_iter=60, rtol=1e-8, precond_pairs=2)
    s.set_numerics(limiter=2)
    del act["lam"]
    torch.cuda.empty_cache()
    p0 = s.params(1, 2)
    fd = []
    for k in range(3):
        h = fd_rel * abs(p0[k])
        J = []
        for sgn in (1, -1):
            p = p0.copy()
            p[k] += sgn * h
            s.set_params(p, 1, 2)
            s.set_state(*base)
            hk = s.iterate(fd_iters)
            J.append(s.wall_heat_flux(1))
            print(f"bench: adjoint check p[{k}] {sgn:+d}h residual {hk[-1].max():.2e}", file=sys.stderr, flush=True)
        fd.append((J[0] - J[1]) / (2 * h))
    s.set_params(p0, 1, 2)
    adj = [float(x) for x in a["dJdp"]]
    return {"check": "dQ_w/dp of the converged sphere (Ma 5, Kn 0.1), p = (T_w, rho_inf, |U_inf|)",
            "n_cells": s.nc, "n_vel": s.nv, "primal_residual": float(hist[-1].max()), "J": a["J"],
            "adjoint_frozen_limiter": {"dJdp": adj, "gmres_iterations": a["iterations"], "restart": 50,
                                       "rel_residual": a["rel_residual"], "seconds": t_adj,
                                       "precond_pairs": 2, "macro_pairs": 20},
            "adjoint_active_limiter": {"dJdp": [float(x) for x in act["dJdp"]], "gmres_iterations": act["iterations"],
                                       "restart": 20, "rel_residual": act["rel_residual"]},
            "central_differences": {"dJdp": [float(x) for x in fd], "h_over_p": fd_rel, "iterations": fd_iters},
            "rel_diff_frozen_vs_fd": [(x - y) / abs(y) for x, y in zip(adj, fd)]}


def _converge(s, tol, max_iter, chunk=100, schedule=None, floor_below=1e-5):
    """Iterate until the residual (largest component) is below tol or, once it is below floor_below, stops
    falling (a rounding floor).  schedule: (iteration, cfl_imp) pairs at multiples of chunk."""
    ramp = dict(schedule or ())
    hist = []
    done = 0
    while done < max_iter:
        if done in ramp:
            s.set_numerics(cfl_imp=ramp[done])
        h = s.iterate(chunk)
        hist.append(h)
        done += chunk
        r = h.max(axis=1)
        if r[-1] < tol or (len(hist) > 2 and r.min() < floor_below and
                           r.min() >= 0.5 * hist[-2].max(axis=1).min()):
            break
    return np.concatenate(hist)


# The two bodies on their hexahedral O-grids: case, description, implicit-step schedule from rest, iteration cap
HEX_WORKLOADS = {
    "sphere_hex": ("sphere Ma 5 Kn 0.1 Tw/Tinf 3 on a hexahedral O-grid (48 384 hexahedra) x 4 140 velocities",
                   None, 1500),
    "capsule_hex": ("capsule Ma 10 Kn 0.01 Tw/Tinf 4.18 on the hexahedral O-grid of the tetrahedral capsule "
                    "(25 272 hexahedra) x 10 568 velocities", "capsule", 3000),
}


def _hex_case(workload):
    from paper_2303_10846_amd.cases import configs
    return configs.sphere_hex_case(seed=0) if workload == "sphere_hex" else configs.capsule_hex_case(seed=0)


def _hex_schedule(workload):
    return CAPSULE_CFL_RAMP if HEX_WORKLOADS[workload][1] == "capsule" else None


def hex_converged(workload="sphere_hex"):
    """A body on its hexahedral O-grid, FP64 and mixed precision, each from rest to the paper's criterion
    (FP64 below 1e-10, Sec. 4.1) or to its rounding floor (mixed), and the mixed fields against the FP64 ones."""
    import torch

    from paper_2303_10846_amd.binding import Solver
    case = _hex_case(workload)
    desc, _, max_iter = HEX_WORKLOADS[workload]
    out = {"workload": desc}
    if _hex_schedule(workload):
        out["cfl_imp_schedule_from_rest"] = [list(x) for x in _hex_schedule(workload)]
    res = {}
    for prec in ("fp64", "mixed"):
        s = Solver(case, precision=prec, device="cuda:0")
        s.init_equilibrium(case["W0"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = _converge(s, 1e-12 if prec == "fp64" else 1e-10, max_iter, schedule=_hex_schedule(workload))
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        r = h.max(axis=1)
        W, _ = s.moments()
        co = s.wall_coefficients(1, 1.0, case["U_inf"], 1.0, A_ref=math.pi * 0.25)
        res[prec] = dict(W=W, Qw=s.wall_heat_flux(1))
        out[prec] = {"iterations": len(r), "residual_last": float(r[-1]), "seconds": t,
                     "ms_per_iteration": 1e3 * t / len(r),
                     "iterations_to_1e-10": int(np.argmax(r < 1e-10)) + 1 if np.any(r < 1e-10) else None,
                     "Qw": res[prec]["Qw"], "Cd": co["Cd"], "CQ": co["CQ"]}
        print(f"bench: {workload} {prec} {len(r)} iterations, residual {r[-1]:.2e}", file=sys.stderr, flush=True)
        del s
        torch.cuda.empty_cache()

    def rho_T(W):
        rho = W[:, 0]
        ke = 0.5 * np.sum(W[:, 1:4] ** 2, axis=1) / rho
        return rho, 0.4 * (W[:, 4] - ke) / (rho * 0.5)

    rm, Tm = rho_T(res["mixed"]["W"])
    rd, Td = rho_T(res["fp64"]["W"])
    err = {"rho": float(np.max(np.abs(rm - rd)) / np.max(np.abs(rd))),
           "T": float(np.max(np.abs(Tm - Td)) / np.max(np.abs(Td))),
           "Qw": abs(res["mixed"]["Qw"] - res["fp64"]["Qw"]) / abs(res["fp64"]["Qw"])}
    out["mixed_vs_fp64_converged"] = dict(err, matched_error=bool(max(err.values()) <= 1e-5))
    return out


def adjoint_check_hex(workload="sphere_hex", fd_rel=1e-6, gmres_iters=600):
    """Discrete adjoint of a converged body on its hexahedral O-grid (FP64, residual below 1e-12) against central
    differences of the converged heat load with step 1e-6 of each parameter, with the limiter differentiated on
    its branch (limiter 1) and with its values stored at the converged state (limiter 3).  The capsule's GMRES
    restart is 40: its Krylov basis (4.3 GB per vector) then takes 190 GB."""
    import torch

    from paper_2303_10846_amd.binding import Solver
    case = _hex_case(workload)
    restart = 60 if workload == "sphere_hex" else 40
    s = Solver(case, precision="fp64", device="cuda:0")
    s.init_equilibrium(case["W0"])
    hist = _converge(s, 1e-13, HEX_WORKLOADS[workload][2], schedule=_hex_schedule(workload))
    print(f"bench: {workload} adjoint check primal residual {hist[-1].max():.3e} after {len(hist)}",
          file=sys.stderr, flush=True)
    base = s.get_state()
    p0 = s.params(1, 2)
    out = {"check": f"dQ_w/dp of the converged {HEX_WORKLOADS[workload][0]}, p = (T_w, rho_inf, |U_inf|)",
           "n_cells": s.nc, "n_vel": s.nv, "primal_iterations": len(hist), "primal_residual": float(hist[-1].max()),
           "gmres_restart": restart}
    for mode, lim in (("active_limiter", 1), ("stored_limiter", 3)):
        s.set_state(*base)
        s.set_params(p0, 1, 2)
        if lim == 3:
            s.freeze_limiter()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a = s.adjoint(1, 2, restart=restart, max_iter=gmres_iters, rtol=1e-10, precond_pairs=2, macro_pairs=20)
        t_adj = time.perf_counter() - t0
        print(f"bench: {workload} adjoint {mode} {a['iterations']} iterations, relative residual "
              f"{a['rel_residual']:.2e}", file=sys.stderr, flush=True)
        del a["lam"]
        torch.cuda.empty_cache()
        fd = []
        for k in range(3):
            h = fd_rel * abs(p0[k])
            J = []
            for sgn in (1, -1):
                p = p0.copy()
                p[k] += sgn * h
                s.set_params(p, 1, 2)
                s.set_state(*base)
                hk = _converge(s, 1e-13, 800)
                J.append(s.wall_heat_flux(1))
                print(f"bench: {workload} adjoint check {mode} p[{k}] {sgn:+d}h residual {hk[-1].max():.2e} "
                      f"after {len(hk)}", file=sys.stderr, flush=True)
            fd.append((J[0] - J[1]) / (2 * h))
        s.set_params(p0, 1, 2)
        if lim == 3:
            s.unfreeze_limiter()
        adj = [float(x) for x in a["dJdp"]]
        out[mode] = {"dJdp_adjoint": adj, "gmres_iterations": a["iterations"], "rel_residual": a["rel_residual"],
                     "adjoint_seconds": t_adj, "dJdp_central_differences": [float(x) for x in fd],
                     "h_over_p": fd_rel, "rel_diff": [(x - y) / abs(y) for x, y in zip(adj, fd)], "J": a["J"]}
    return out


# Implicit-step schedule of a capsule run that starts from a converged macroscopic field (another DVS's)
CAPSULE_WARM_RAMP = ((0, 10.0), (100, 30.0), (300, 100.0))


def capsule_dvs_study(iters, warm_iters=1000):
    """The capsule's wall coefficients against the DVS.  The timed workload's set (C1) runs from rest with the
    schedule of the convergence run; each other set starts from the equilibrium of C1's converged W and runs
    `warm_iters` iterations (a coarse set from rest does not survive the bow shock's formation at cfl_imp = 1:
    its state turns non-physical).  Relative differences against C1."""
    import torch

    from paper_2303_10846_amd.binding import CisError, Solver
    from paper_2303_10846_amd.cases import configs, dvs
    case = configs.capsule_case(seed=0)
    T0 = dvs.total_temperature(1.0, case["mach"])
    rtop = math.sqrt(0.5 * max(T0, case["T_w"]))

    def run(c, W0, sched, n_it, name):
        s = Solver(c, precision="mixed", device="cuda:0")
        s.init_equilibrium(W0)
        ramp = dict(sched)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, res = 0, None
        while done < n_it:
            if done in ramp:
                s.set_numerics(cfl_imp=ramp[done])
            try:
                h = s.iterate(100)
            except CisError as e:
                print(f"bench: capsule dvs study {name} stopped at {done}: {e}", file=sys.stderr, flush=True)
                return s, None, done, time.perf_counter() - t0
            done += 100
            res = float(h[-1].max())
            print(f"bench: capsule dvs study {name} {done} iterations, residual {res:.3e}", file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        return s, res, done, time.perf_counter() - t0

    rows = []
    s, res, done, t = run(case, case["W0"], CAPSULE_CFL_RAMP, iters, "C1")
    W_ref, _ = s.moments()
    rows.append(dict(name="C1", radius_over_sqrt_RT0=5.0, n_vel=len(case["u"]), start="rest", iterations=done,
                     residual=res, ms_per_iter=1e3 * t / max(done, 1), **_coefficients(s, case)))
    del s
    torch.cuda.empty_cache()
    for name, factor, target in CAPSULE_DVS_STUDY:
        u, w = dvs.paper_unstructured_dvs(case["U_inf"], 1.0, case["T_w"], case["mach"], factor, target=target)
        c = dict(case, u=u, w=w)
        print(f"bench: capsule dvs study {name}: radius {factor} sqrt(R T0), {len(u)} velocities", file=sys.stderr,
              flush=True)
        s, res, done, t = run(c, W_ref, CAPSULE_WARM_RAMP, warm_iters, name)
        row = dict(name=name, radius_over_sqrt_RT0=factor, n_vel=len(u), start="C1's converged W",
                   ball_volume_covered=float(w.sum() / (4.0 / 3.0 * math.pi * (factor * rtop) ** 3)),
                   iterations=done, residual=res, ms_per_iter=1e3 * t / done if done else None)
        if res is not None:
            row.update(_coefficients(s, c))
            row["rel_diff_vs_C1"] = {k: (row[k] - rows[0][k]) / abs(rows[0][k]) for k in ("Cd", "CQ", "Cp_max", "Ch_max")}
        rows.append(row)
        del s
        torch.cuda.empty_cache()
    return {"study": "DVS size and extent, capsule Ma 10 Kn 0.01 Tw/Tinf 4.18", "n_cells": len(case["mesh"]["tets"]),
            "precision": "mixed", "A_ref": "pi D^2 / 4", "cfl_imp_schedule_from_rest": [list(x) for x in CAPSULE_CFL_RAMP],
            "cfl_imp_schedule_warm": [list(x) for x in CAPSULE_WARM_RAMP], "sets": rows}


# Implicit-step schedule of the capsule's convergence run: iteration from which each cfl_imp applies.  Ma 10 from
# rest needs a small implicit step until the bow shock has formed; afterwards the step grows.
CAPSULE_CFL_RAMP = ((0, 1.0), (800, 3.0), (1100, 10.0), (1400, 30.0), (1700, 100.0))


def capsule_converge(iters):
    """The Ma 10 capsule (mixed precision) from rest to its converged coefficients, with the cfl_imp schedule
    above: residual, C_d, heat-load coefficient C_Q and C_l every 100 iterations."""
    import torch

    from paper_2303_10846_amd.binding import Solver, wall_coefficients
    from paper_2303_10846_amd.cases import configs
    case = configs.capsule_case(seed=0)
    s = Solver(case, precision="mixed", device="cuda:0")
    s.init_equilibrium(case["W0"])
    ramp = dict(CAPSULE_CFL_RAMP)
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < iters:
        if done in ramp:
            s.set_numerics(cfl_imp=ramp[done])
        h = s.iterate(100)
        done += 100
        co = wall_coefficients(s.wall_loads(1), 1.0, case["U_inf"], 1.0, 0.5, A_ref=math.pi * 0.25)
        row = dict(iteration=done, seconds=time.perf_counter() - t0, residual=float(h[-1].max()), Cd=co["Cd"],
                   CQ=float(co["CQ"]), Cl=co["Cl"])
        hist.append(row)
        print(f"bench: capsule {done} iterations, residual {row['residual']:.3e}, Cd {row['Cd']:.6f}, "
              f"CQ {row['CQ']:.6f}", file=sys.stderr, flush=True)
    return {"run": "capsule Ma 10 Kn 0.01 Tw/Tinf 4.18 from rest, mixed precision, A_ref = pi D^2 / 4",
            "n_cells": s.nc, "n_vel": s.nv, "cfl_imp_schedule": [list(x) for x in CAPSULE_CFL_RAMP],
            "history": hist}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precision", choices=["both", "mixed", "fp64"], default="both")
    ap.add_argument("--sweeps", type=int, nargs=2, default=None, metavar=("N_MACRO", "N_MICRO"),
                    help="forward + backward pairs of the macro and micro sweeps (default 40 2, the paper's "
                         "PR-SGS setting; 1 1 is LU-SGS)")
    ap.add_argument("--converge-iters", type=int, default=600,
                    help="iterations (from rest) after which the two precisions' fields are compared")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (calibrates HBM byte counters)")
    ap.add_argument("--workload", choices=["sphere", "capsule", "sphere_hex", "capsule_hex"], default="sphere",
                    help="sphere (the headline workload), the Ma 10 capsule (303k tets x 10.6k velocities, "
                         "mixed precision only: its FP64 state does not fit one GPU), or either body on its "
                         "hexahedral O-grid (timed, and with --adjoint-check the adjoint at its converged state)")
    ap.add_argument("--no-hex-capsule", action="store_true",
                    help="leave out the converged hexahedral-capsule block of the default line")
    ap.add_argument("--no-hex", action="store_true",
                    help="leave out the converged hexahedral-sphere block of the default line")
    ap.add_argument("--dvs-study", type=int, default=0, metavar="ITERS",
                    help="instead of timing, run the sphere with six DVS sets for ITERS iterations each and print "
                         "the wall coefficients against the DVS")
    ap.add_argument("--adjoint-check", action="store_true",
                    help="instead of timing, solve the sphere's discrete adjoint and compare dQ_w/dp with central "
                         "differences of the converged heat load")
    ap.add_argument("--capsule-converge", type=int, default=0, metavar="ITERS",
                    help="instead of timing, run the capsule from rest for ITERS iterations (a multiple of 100) "
                         "and print its residual and wall coefficients every 100 iterations")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the DVS-sharded multi-GPU path is a design, not code); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe_mb:
        import torch
        n = args.copy_probe_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.mul(a, 2.0, out=b)   # one elementwise kernel: reads n floats, writes n floats
        torch.cuda.synchronize()
        print(f"bench: copy probe {args.copy_probe_mb} MiB read + {args.copy_probe_mb} MiB written",
              file=sys.stderr, flush=True)
        del a, b
    if args.capsule_converge:
        print(json.dumps(capsule_converge(args.capsule_converge)))
        return
    if args.adjoint_check:
        print(json.dumps(adjoint_check_hex(args.workload) if args.workload in HEX_WORKLOADS else adjoint_check()))
        return
    if args.dvs_study:
        print(json.dumps(dvs_study(args.dvs_study, args.workload)))
        return
    from paper_2303_10846_amd.cases import configs
    if args.workload == "capsule":
        if args.precision == "fp64":
            print("bench.py: the capsule's FP64 state does not fit one GPU; use --precision mixed", file=sys.stderr)
            sys.exit(2)
        args.precision = "mixed"
        args.converge_iters = 0
    if args.workload in HEX_WORKLOADS:
        case = _hex_case(args.workload)
    else:
        case = configs.sphere_case(seed=0) if args.workload == "sphere" else configs.capsule_case(seed=0)
    if args.sweeps:
        case["num"] = dict(case["num"], n_macro=args.sweeps[0], n_micro=args.sweeps[1])
    mesh = case["mesh"]
    print(f"bench: {case['name']} cells={len(mesh['tets'] if 'tets' in mesh else mesh['cells'])} nv={len(case['u'])}",
          file=sys.stderr, flush=True)
    res = {}
    for prec in (["mixed", "fp64"] if args.precision == "both" else [args.precision]):
        print(f"bench: timing {prec}", file=sys.stderr, flush=True)
        res[prec] = run_path(case, prec, args.steps, args.warmup, args.converge_iters, args.workload)
        print(f"bench: {prec} {res[prec]['ms_per_step']:.2f} ms/iter", file=sys.stderr, flush=True)
    main_key = "mixed" if "mixed" in res else "fp64"
    r = res[main_key]
    line = {
        "metric": "cell-velocity updates/s per implicit iteration",
        "value": r["value"], "unit": "cell-velocity updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if main_key == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": ("sphere Ma 5 Kn 0.1 Tw/Tinf 3, graded tets x unstructured DVS, from rest"
                                if args.workload == "sphere" else
                                "capsule Ma 10 Kn 0.01 Tw/Tinf 4.18, graded tets x unstructured DVS, from rest"
                                if args.workload == "capsule" else
                                HEX_WORKLOADS[args.workload][0] + ", from rest"),
                   "n_cells": r["n_cells"], "n_faces": r["n_faces"], "n_vel": r["n_vel"], "pairs": r["pairs"],
                   "precision": main_key, "n_macro_sweeps": case["num"]["n_macro"],
                   "n_micro_sweeps": case["num"]["n_micro"]},
        "roofline": r["roofline"],
        "roofline_iteration": r["roofline_iteration"],
        "stages": r["stages"],
    }
    if r["roofline_sweep"]:
        line["roofline_micro_sweep"] = r["roofline_sweep"]
    if args.converge_iters:
        line["convergence"] = {"iterations": r["iterations"], "residual_last": r["residual_last"],
                               "iterations_to_residual": r["iterations_to"], "Qw": r["Qw"]}
    if "fp64" in res and main_key != "fp64":
        f = res["fp64"]
        line["fp64"] = {"value": f["value"], "ms_per_step": f["ms_per_step"], "roofline": f["roofline"],
                        "roofline_micro_sweep": f["roofline_sweep"], "roofline_iteration": f["roofline_iteration"],
                        "stages": f["stages"]}
        Wm, Wd = r["W"], f["W"]

        def rho_T(W):
            rho = W[:, 0]
            ke = 0.5 * np.sum(W[:, 1:4] ** 2, axis=1) / rho
            return rho, 0.4 * (W[:, 4] - ke) / (rho * 0.5)

        rm, Tm = rho_T(Wm)
        rd, Td = rho_T(Wd)
        err = {"rho": float(np.max(np.abs(rm - rd)) / np.max(np.abs(rd))),
               "T": float(np.max(np.abs(Tm - Td)) / np.max(np.abs(Td))),
               "Qw": abs(r["Qw"] - f["Qw"]) / abs(f["Qw"])}
        basis = ("fields after the same number of iterations from rest (residuals beside), mixed against the FP64 "
                 "GPU run")
        if args.workload == "sphere":
            basis += (", both at the limiter plateau of the tetrahedral mesh; converged fields: converged_hex_sphere "
                      "and converged_hex_capsule")
        line["mixed_vs_fp64"] = dict(err, basis=basis,
                                     iterations=r["iterations"], residual_mixed=r["residual_last"],
                                     residual_fp64=f["residual_last"], Qw_fp64=f["Qw"],
                                     matched_error=bool(max(err.values()) <= 1e-5),
                                     iterations_to_residual_mixed=r["iterations_to"],
                                     iterations_to_residual_fp64=f["iterations_to"])
    if args.workload == "sphere" and args.converge_iters and not args.no_hex:
        print("bench: hexahedral sphere to convergence", file=sys.stderr, flush=True)
        line["converged_hex_sphere"] = hex_converged("sphere_hex")
    if args.workload == "sphere" and args.converge_iters and not args.no_hex_capsule:
        print("bench: hexahedral capsule to convergence", file=sys.stderr, flush=True)
        line["converged_hex_capsule"] = hex_converged("capsule_hex")
    if not args.no_cpu and args.workload == "sphere":
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(case)
    elif not args.no_cpu:
        # the other workloads take the oracle's per-pair rate on the sphere workload, labelled as an extrapolation
        # (the capsule's FP64 oracle state does not fit the host's memory)
        print("bench: cpu baseline (oracle on the sphere workload, extrapolated)", file=sys.stderr, flush=True)
        cb = cpu_baseline(configs.sphere_case(seed=0))
        cb["kind"] = "oracle, extrapolated"
        cb["extrapolation"] = (f"the oracle's per-pair rate on the sphere workload applied to this workload's "
                               f"{r['pairs']:.3g} pairs: {r['pairs'] / cb['value']:.1f} s per iteration")
        line["cpu_baseline"] = cb
    print(json.dumps(line))


if __name__ == "__main__":
    main()
