"""The rocprofv3 summary tool on synthetic counter files (no GPU): byte calibration and VALU issue time."""
import csv
import os

from paper_2303_10846_amd import prof_summary

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_counters_calibrate_against_the_copy_probe(tmp_path):
    probe = "void at::native::vectorized_elementwise_kernel<4, std::array<char*, 2ul> >(int)"
    kern = "void cis::k_micro_sweep_vec<4>(cis::Dev, cis::Bufs, cis::Work, long, long, int)"
    # the probe moves 1 GiB each way; FETCH_SIZE reads it as half (two rows per dispatch split the value)
    _write(tmp_path / "fetch", [(1, probe, "FETCH_SIZE", 262144.0), (1, probe, "FETCH_SIZE", 262144.0),
                                (2, kern, "FETCH_SIZE", 1000.0), (3, kern, "FETCH_SIZE", 3000.0)])
    _write(tmp_path / "write", [(1, probe, "WRITE_SIZE", 1048576.0), (2, kern, "WRITE_SIZE", 500.0),
                                (3, kern, "WRITE_SIZE", 700.0)])
    out = tmp_path / "c.txt"
    prof_summary.counters(str(tmp_path / "fetch"), str(tmp_path / "write"), str(out), "k_micro_sweep_vec<4>",
                          1024, "cmd PMC")
    c = prof_summary.read_counters(str(out))
    assert float(c["fetch_scale"]) == 2.0 and float(c["write_scale"]) == 1.0
    assert float(c["hbm_read_bytes_per_dispatch"]) == 2000.0 * 1024 * 2.0    # mean 2000 KiB, scaled by 2
    assert float(c["hbm_write_bytes_per_dispatch"]) == 600.0 * 1024
    assert c["source_sha256"] == prof_summary.source_hash()


def test_sq_valu_issue_time(tmp_path):
    kern = "void cis::k_face<float, true>(cis::Dev, cis::Bufs, cis::Work)"
    # 2 dispatches of 2.4e9 / 4 * 1024 * 1e-3 VALU wavefront instructions each: 1000 us of issue at 2.4 GHz
    n = 2.4e9 * 1e-3 * 1024 / 4
    _write(tmp_path / "sq", [(1, kern, "SQ_INSTS_VALU", n), (2, kern, "SQ_INSTS_VALU", n),
                             (1, kern, "SQ_WAVES", 1000.0), (2, kern, "SQ_WAVES", 1000.0)])
    out = tmp_path / "sq.txt"
    prof_summary.sq(str(tmp_path / "sq"), str(out), "cmd", ["k_face<"])
    text = open(out).read()
    assert "valu_issue_us: 1000.0" in text
    assert f"valu_per_wave: {n / 1000.0:.1f}" in text
