"""Host logic of bench.py (CPU): the HBM-traffic record is used only for the
kernel sources it was measured on, the committed record adds up, and the
roofline object is formed as documented (frac = achieved / 8 TB/s for the
CG iteration as a whole, the dominant kernel the longest one, traffic over
the per-iteration algorithmic bytes)."""
import os
import shutil

import pytest

import bench

RECORD = os.path.join(bench.ROOT, "profiles", "traffic.txt")


def read_record(path):
    rec = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            rec[k.strip()] = v.strip()
    return rec


def copy_tree(dst):
    csrc = os.path.join(dst, "paper_1808_06381_amd", "csrc")
    os.makedirs(csrc)
    for f in ("cg.hip", "sim_dev.h"):
        shutil.copy(os.path.join(bench.ROOT, "paper_1808_06381_amd", "csrc", f), csrc)
    os.makedirs(os.path.join(dst, "profiles"))


def test_traffic_record_keyed_to_the_kernel_sources(tmp_path, monkeypatch):
    copy_tree(str(tmp_path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    sha = bench.kernel_source_sha()
    lines = ["# test record", f"source_sha={sha}", "workload=c5_single_n8e6", "form=learned",
             "k_cg_vec.traffic_bytes_per_launch=100", "cg_iteration.traffic_bytes=300",
             "cg_iteration.algorithmic_bytes=200"]
    with open(tmp_path / "profiles" / "traffic.txt", "w") as f:
        f.write("\n".join(lines) + "\n")
    t = bench.read_traffic("c5_single_n8e6", "learned")
    assert t == dict(bytes_per_iteration=300.0, algorithmic_bytes_per_iteration=200.0,
                     k_cg_vec=100.0)
    assert bench.read_traffic("c5_single_n8e6", "plain") is None      # another form
    assert bench.read_traffic("single_n1e6_x3", "learned") is None     # another workload
    # any edit of the CG sources (a comment too) retires the record
    with open(tmp_path / "paper_1808_06381_amd" / "csrc" / "cg.hip", "a") as f:
        f.write("// edited\n")
    assert bench.kernel_source_sha() != sha
    assert bench.read_traffic("c5_single_n8e6", "learned") is None


def test_committed_traffic_record_adds_up():
    rec = read_record(RECORD)
    fs, ws = float(rec["copy_fetch_scale"]), float(rec["copy_write_scale"])
    # the copy calibration: FETCH_SIZE counts about half of a copy's reads
    assert 1.9 < fs < 2.1 and 0.95 < ws < 1.05
    kernels = ("k_cg_vec", "k_cg_spmv", "k_cg_apply", "k_cg_finish", "k_cg_reduce1")
    # the counters are stored to 0.001 KiB, the bytes to the unit
    tol = 0.0005 * 1024 * (fs + ws) + 0.5
    total = 0.0
    for k in kernels:
        want = (float(rec[f"{k}.fetch_kib"]) * 1024 * fs + float(rec[f"{k}.write_kib"]) * 1024 * ws)
        got = float(rec[f"{k}.traffic_bytes_per_launch"])
        assert got == pytest.approx(want, rel=1e-6, abs=tol), k
        total += got
    assert float(rec["cg_iteration.traffic_bytes"]) == pytest.approx(total, rel=1e-9,
                                                                     abs=0.5 * len(kernels))
    # at least the formula's algorithmic bytes (the single-reduction CG moves
    # the extra vectors s and w besides); re-reads would push it past 1.5x
    ratio = float(rec["cg_iteration.traffic_bytes"]) / float(rec["cg_iteration.algorithmic_bytes"])
    assert 1.0 <= ratio < 1.5


def test_iteration_roofline_object():
    k = 5.5
    n = 8_000_000
    alg = (12 * (k + 1) + 4 + 200 + 12 * (k + 1) + 4) * n   # learned form
    us = 720.0
    r = dict(rows=dict(mean_offdiag_per_row=k),
             kernels=dict(cg_iteration=dict(gbs=alg / us / 1e3, bytes_per_launch=alg, mean_us=us,
                                            launches=50),
                          k_cg_vec=dict(gbs=6000.0, bytes_per_launch=1.6e9, mean_us=266.0),
                          k_cg_spmv=dict(gbs=4500.0, bytes_per_launch=1.0e9, mean_us=222.0),
                          k_cg_apply=dict(gbs=4000.0, bytes_per_launch=0.8e9, mean_us=200.0)))
    traffic = dict(bytes_per_iteration=1.28 * alg, algorithmic_bytes_per_iteration=alg,
                   k_cg_vec=1.7e9)
    out = bench.iteration_roofline(r, 5150.0, traffic)
    assert out["bound"] == "hbm" and out["peak"] == 8000.0 and out["unit"] == "GB/s"
    assert out["frac"] == pytest.approx(alg / us / 1e3 / 8000.0, abs=1e-4)
    assert out["achieved"] == pytest.approx(alg / us / 1e3, abs=0.1)
    assert out["traffic"] == traffic["bytes_per_iteration"]
    assert out["traffic_over_algorithmic"] == pytest.approx(1.28, abs=1e-4)
    assert out["dominant_kernel"]["kernel"] == "k_cg_vec"
    assert out["dominant_kernel"]["traffic"] == 1.7e9
    assert out["frac_of_copy_probe"] == pytest.approx(alg / us / 1e3 / 5150.0, abs=1e-4)
    # without a current counter record the traffic fields are null
    out2 = bench.iteration_roofline(r, 5150.0, None)
    assert out2["traffic"] is None and out2["dominant_kernel"]["traffic"] is None
    assert "traffic_over_algorithmic" not in out2
