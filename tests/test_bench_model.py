"""The benchmark's byte model, sweep counting and output contract (no GPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _sequence(off, n_pairs):
    """Colour order of n_pairs forward + backward passes, a colour that follows itself relaxed once."""
    seq = []
    n = len(off) - 1
    for _ in range(n_pairs):
        for c in list(range(n)) + list(range(n - 1, -1, -1)):
            if off[c + 1] > off[c] and (not seq or seq[-1] != c):
                seq.append(c)
    return seq


@pytest.mark.parametrize("off,pairs", [([0, 3, 5, 9], 2), ([0, 4, 4, 10], 1), ([0, 7], 3), ([0, 2, 6, 7, 12], 40)])
def test_sweep_cells_counts_the_deduplicated_relaxations(off, pairs):
    seq = _sequence(off, pairs)
    want = sum(off[c + 1] - off[c] for c in seq)
    assert bench.sweep_cells(off, pairs) == want
    # three colours, two pairs: 0 1 2 1 0 1 2 1 0 (the last colour once at each turn, the first at the middle)
    if off == [0, 3, 5, 9] and pairs == 2:
        assert seq == [0, 1, 2, 1, 0, 1, 2, 1, 0]


def test_stage_bytes_model():
    nc, nf, nv, es, mc = 10, 22, 7, 4, 30
    sb = bench.stage_bytes(nc, nf, nv, es, mc)
    assert sb["recon"] == (2 * nc + 2 * nf) * nv * es
    assert sb["face"] == 4 * nf * nv * es
    assert sb["residual"] == (2 * nf + 4 * nc) * nv * es
    assert sb["micro"] == 6 * mc * nv * es
    assert sb["update"] == 6 * nc * nv * es


def test_scope_table_byte_model():
    nc, nv, es, mc = 10, 7, 4, 30
    mb = bench.model_bytes(nc, nv, es, mc)
    assert mb["face"] == 4 * nc * nv * es           # face pass: read phi (G, R), write F (G, R)
    assert mb["residual"] == 6 * nc * nv * es
    assert mb["micro"] == 6 * mc * nv * es
    assert mb["update"] == 6 * nc * nv * es
    # four full half-sweeps (mc = 4 nc) give the model's 40 words per (cell, velocity)
    full = bench.model_bytes(nc, nv, es, 4 * nc)
    assert sum(full.values()) == bench.MODEL_WORDS_PER_ITER * nc * nv * es


def test_roofline_carries_the_contract_keys():
    r = bench.roofline("micro", "mixed", 9.0e9, 2.0, 9.0, workload="no-such-workload")
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["traffic"] is None                                   # no committed counters for this workload
    assert abs(r["achieved"] - 9.0e9 / 9 / (2.0e-3 / 9) / 1e9) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12
    r2 = bench.roofline("face", "mixed", 3.0e9, 3.0, 1.0, workload="no-such-workload", kernel_bytes_iter=6.0e9)
    assert abs(r2["achieved"] - 1000.0) < 1e-9 and abs(r2["kernel_model"]["achieved"] - 2000.0) < 1e-9


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


class _FakeSolver:
    """Stands in for a Solver in the convergence loop: the residual history follows a given function of the
    iteration count, and every implicit-step change is recorded."""

    def __init__(self, residual_of):
        self.residual_of = residual_of
        self.done = 0
        self.cfl = []

    def set_numerics(self, **kw):
        self.cfl.append((self.done, kw["cfl_imp"]))

    def iterate(self, n):
        import numpy as np
        r = np.array([self.residual_of(self.done + k + 1) for k in range(n)])
        self.done += n
        return np.repeat(r[:, None], 6, axis=1)


def test_converge_stops_at_tol_and_applies_the_schedule():
    s = _FakeSolver(lambda it: 10.0 ** (-it / 100.0))
    h = bench._converge(s, 1e-8, 3000, schedule=((0, 1.0), (300, 3.0), (900, 10.0)))
    # below 1e-8 first at iteration 801, checked at the end of each 100-iteration chunk
    assert len(h) == 900 and h[-1].max() < 1e-8
    assert s.cfl == [(0, 1.0), (300, 3.0)]


def test_converge_stops_at_a_rounding_floor_only_below_floor_below():
    # a slow transient above 1e-5 (falls by less than half per chunk) must not stop the loop; a floor at 2e-6 does
    def res(it):
        if it <= 500:
            return 0.1 * 0.9 ** (it / 100.0)
        return max(2e-6, 0.1 * 0.9 ** 5 * 10.0 ** (-(it - 500) / 100.0))
    s = _FakeSolver(res)
    h = bench._converge(s, 1e-10, 5000)
    r = h.max(axis=1)
    assert r[-1] == 2e-6 and len(h) < 5000
    assert len(h) > 500


def test_hex_workloads_take_the_capsule_schedule():
    assert bench._hex_schedule("capsule_hex") == bench.CAPSULE_CFL_RAMP
    assert bench._hex_schedule("sphere_hex") is None
    assert set(bench.HEX_WORKLOADS) == {"sphere_hex", "capsule_hex"}
