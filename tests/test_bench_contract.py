"""Host checks of bench.py's contract: more than one GPU is refused, and the
committed counter records it reads (HBM traffic of the D1Q3 step, VALU count
of the D2Q9 step) are arithmetically consistent with their raw counters."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


# sites per launch of each counted workload: L = 2^24, L = 2^27 (one step
# per launch, and in tiles), and the 1024-replica manifest (one step per
# launch, and whole replicas per block)
TRAFFIC_SITES = {"plain": 1 << 24, "probe": 1 << 27, "batched": 137_671_148,
                 "probe_blocked": 1 << 27, "batched_blocked": 137_671_148}


@pytest.mark.parametrize("which", sorted(TRAFFIC_SITES))
def test_traffic_record_follows_from_its_counters(which):
    d = json.load(open(bench.TRAFFIC_FILES[which]))
    cal = d["copy_calibration"]
    # the calibration copy moves a known number of bytes each way
    assert cal["fetch_factor"] == pytest.approx(cal["bytes_read"] / 1024 / cal["fetch_size_kib"])
    assert cal["write_factor"] == pytest.approx(cal["bytes_written"] / 1024 / cal["write_size_kib"])
    want = 1024 * (d["fetch_size_kib_per_dispatch"] * cal["fetch_factor"] +
                   d["write_size_kib_per_dispatch"] * cal["write_factor"])
    assert d["bytes_per_launch"] == pytest.approx(want, rel=1e-9)
    # 12 bytes per site update, every site once per step of the launch
    assert d["algorithmic_bytes_per_launch"] == (bench.BYTES_PER_SITE_UPDATE * TRAFFIC_SITES[which]
                                                 * d.get("steps_per_launch", 1))
    assert d["ratio_to_algorithmic"] == pytest.approx(d["bytes_per_launch"] /
                                                      d["algorithmic_bytes_per_launch"])
    assert len(d["kernel_sha256_16"]) == 16
    assert [os.path.basename(p) for p in bench.KERNEL_SRCS] == d["kernel_sources"]


def test_batched_manifest_size():
    import synth
    assert int(sum(synth.replica_manifest()["L"])) == TRAFFIC_SITES["batched"]


def test_valu_record_follows_from_its_counters():
    v = json.load(open(bench.D2Q9_VALU_FILE))
    assert v["valu_insts_per_wave"] == pytest.approx(
        v["sq_insts_valu_per_dispatch"] / v["sq_waves_per_dispatch"], abs=0.01)
    # one wave per 64 sites of the 4096 x 4096 lattice
    assert v["sq_waves_per_dispatch"] == 4096 * 4096 // 64
    assert [os.path.basename(p) for p in bench.D2Q9_SRCS] == v["kernel_sources"]


def test_valu_issue_peak():
    # 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles, 2.4 GHz
    assert bench.VALU_PEAK_G == pytest.approx(614.4)


@pytest.mark.parametrize("which", sorted(TRAFFIC_SITES))
def test_valu_issue_fraction_from_the_record(which):
    d = json.load(open(bench.TRAFFIC_FILES[which]))
    # 256 persistent blocks of 16 waves
    assert d["sq_waves_per_dispatch"] == 4096
    assert d["sq_insts_valu_per_dispatch"] > 0
    K = d.get("steps_per_launch", 1)
    if d["kernel_sha256_16"] == bench.kernel_hash():
        t = 1e-3
        assert bench.valu_issue_frac(which, t, K) == pytest.approx(
            d["sq_insts_valu_per_dispatch"] / (bench.VALU_PEAK_G * 1e9) / t)
        assert bench.valu_issue_frac(which, t, K + 1) is None
    else:
        assert bench.valu_issue_frac(which, 1e-3, K) is None
