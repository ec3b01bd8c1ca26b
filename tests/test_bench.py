"""Host-side pieces of the benchmark: its byte models, the committed counter
summaries it reads, and its one-GPU contract (no device needed)."""

import json
import os
import subprocess
import sys

import pytest

import bench
import problems

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_compulsory_bytes_per_zone_cycle():
    # torus 288 x 128 x 128: 320 B of state traffic + 150 doubles of 2D
    # geometry per (x1, x2) column and substep over 128 planes
    prm = dict(coords=problems.KERR_FMKS, n3=128, precision=problems.FP64)
    assert bench.compulsory_bytes_per_zone_cycle(prm) == 338.75
    # Minkowski: no geometry
    assert bench.compulsory_bytes_per_zone_cycle(dict(prm, coords=problems.MINKOWSKI_CART)) == 320.0
    # Cartesian Kerr-Schild: every zone's connection and floor scales (42
    # values) per substep, the metric evaluated in closed form; in mixed
    # precision the three float face tables (22 values each) as well
    cks = dict(coords=problems.KERR_CKS, n3=168, precision=problems.FP64)
    assert bench.compulsory_bytes_per_zone_cycle(cks) == 320 + 2 * 42 * 8 == 992
    assert bench.compulsory_bytes_per_zone_cycle(dict(cks, precision=problems.MIXED)) == 320 + 2 * (42 * 8 + 3 * 22 * 4)


def test_split_design_bytes_count_the_face_fluxes():
    prm, _ = problems.fm_torus(n1=64, n2=32, n3=16)
    zones = 64 * 32 * 16
    upd = bench.split_design_bytes("update", prm, False)
    # 21 flux values, 96 B of states on average, 64 B written, a flag byte, the 2D table
    assert upd == zones * (21 * 8 + 96 + 64 + 1) + 64 * 8 * 64 * 32
    assert bench.split_design_bytes("update", prm, True) == zones * (21 * 4 + 96 + 64 + 1) + 64 * 8 * 64 * 32
    with pytest.raises(KeyError):
        bench.split_design_bytes("ghosts", prm, False)


def test_committed_counter_summaries_have_the_fields_bench_reads():
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as f:
        hbm = json.load(f)
    assert len(hbm["library_hash"]) == 16
    for workload, rec in hbm["workloads"].items():
        for cls in ("sweeps", "update"):
            k = rec["kernels"][cls]
            assert k["bytes_per_launch"] > 0 and k["launches_per_step"] == 2, (workload, cls)
        assert rec["fetch_scale"] > 1.0 and rec["write_scale"] > 0.5
    with open(os.path.join(ROOT, "profiles", "valu_flops.json")) as f:
        valu = json.load(f)
    assert valu["library_hash"] == hbm["library_hash"]
    for workload, rec in valu["workloads"].items():
        for cls in ("sweeps", "update"):
            assert rec[cls]["fp64"] >= 0 and rec[cls]["fp32"] >= 0


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_arithmetic_ceiling_of_the_hbm_fraction():
    zones, per_zc = 1000, 320.0
    balance = bench.FP64_PEAK / bench.HBM_PEAK
    # exactly the machine balance: a step at the FP64 peak moves its bytes at the HBM peak
    at_balance = bench.arithmetic_ceiling(balance * zones * per_zc, zones, per_zc, 1.0)
    assert abs(at_balance["step_compulsory_frac_ceiling"] - 1.0) < 1e-12
    # twice the balance: half the HBM peak at best
    twice = bench.arithmetic_ceiling(2 * balance * zones * per_zc, zones, per_zc, 1.0)
    assert abs(twice["step_compulsory_frac_ceiling"] - 0.5) < 1e-12
    assert abs(twice["flop_per_compulsory_byte"] - 2 * balance) < 1e-9
    # less work than the balance: HBM bound, the ceiling stays 1
    assert bench.arithmetic_ceiling(0.1 * zones * per_zc, zones, per_zc, 1.0)["step_compulsory_frac_ceiling"] == 1.0
    # the measured FP64 fraction: flops over the step time against the vector peak
    r = bench.arithmetic_ceiling(bench.FP64_PEAK * 1e-3, zones, per_zc, 4e-3)
    assert abs(r["step_fp64_frac"] - 0.25) < 1e-12


def test_timed_kernel_classes_cover_the_dominant_candidates():
    """Inside the timed region the bench brackets only TIMED_KERNELS with
    events; the dominant kernel is chosen among the face fluxes and the update,
    so both must be timed there, and every name must be a library class."""
    import paper_2110_10191_amd as g
    assert set(bench.TIMED_KERNELS) == {"sweeps", "update"}
    assert set(bench.TIMED_KERNELS) <= set(g.KERNELS)
    mask = 0
    for name in bench.TIMED_KERNELS:
        mask |= 1 << g.KERNELS[name]
    assert 0 < mask < 1 << (max(g.KERNELS.values()) + 1)
