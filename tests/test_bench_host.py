"""Host logic of the benchmark (CPU only): the one-GPU refusal, the algorithmic byte
model the roofline divides by, the sweep's lattice sizes, and the internal arithmetic of
the committed HBM-traffic record."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_stored_diffusion_bytes_per_apply():
    """x read and y written once (8 B per dof each), six FP64 values of D per point on
    (p+2)^3 points, and the int32 element-to-dof map: at p = 1 on the sweep's 214^3
    lattice (9,938,375 dofs) that is the 13,173,870,832 B per launch the roofline quotes."""
    n = bench.lattice_size(1, 1e7)
    ne, nd = n ** 3, (n + 1) ** 3
    assert (n, nd) == (214, 9938375)
    expect = 16 * nd + ne * 27 * 6 * 8 + ne * 8 * 4
    assert bench.algorithmic_bytes("diffusion", 1, ne, nd) == expect == 13173870832
    # mass stores one value per point
    assert bench.algorithmic_bytes("mass", 1, ne, nd) == 16 * nd + ne * 27 * 8 + ne * 8 * 4


@pytest.mark.parametrize("p", range(1, 9))
def test_sweep_lattices_hold_about_ten_million_dofs(p):
    n = bench.lattice_size(p, 1e7)
    assert 0.85e7 < (n * p + 1) ** 3 < 1.15e7


def test_traffic_record_arithmetic():
    """The record's bytes per launch are its counters (KiB per dispatch, apply plus its
    y-init) scaled by the calibration factors, which are the copy's known bytes over its
    counters; the record is used only for the sources it was taken on."""
    with open(os.path.join(ROOT, "profiles", "pa_apply_diffusion_p1_traffic.json")) as fh:
        rec = json.load(fh)
    cal = rec["calibration"]
    assert abs(cal["fetch_scale"] - cal["copy_bytes"] / (cal["copy_fetch_kib"] * 1024)) < 1e-12
    assert abs(cal["write_scale"] - cal["copy_bytes"] / (cal["copy_write_kib"] * 1024)) < 1e-12
    f = rec["fetch_kib_per_dispatch"]
    w = rec["write_kib_per_dispatch"]
    fetch = (f["apply"] + f["init"]) * 1024 * cal["fetch_scale"]
    write = (w["apply"] + w["init"]) * 1024 * cal["write_scale"]
    assert abs(fetch - rec["fetch_bytes_per_launch"]) < 1e-6 * fetch
    assert abs(write - rec["write_bytes_per_launch"]) < 1e-6 * write
    assert rec["traffic_bytes_per_launch"] == round(fetch + write)
    got = bench.recorded_traffic(1)
    if rec["source_hash"] == bench.apply_source_hash():
        assert got == rec["traffic_bytes_per_launch"]
    else:
        assert got is None
