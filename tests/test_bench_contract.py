"""Host-side checks of the measurement code in bench.py: the traffic record is
used only while every source file it names is unchanged, the pair work counts
the z pass on the eps sphere's occupied (x, y) columns, and more than one GPU is
refused."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _record(tmp, sources, fetch=1000.0, write=500.0, fscale=2.0, wscale=1.0):
    rec = {"pair_plane": {"kernel": "k", "dispatches": 1,
                          "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write,
                          "fetch_scale": fscale, "write_scale": wscale, "sources": sources}}
    prof = tmp / "profiles"
    prof.mkdir()
    (prof / "traffic_cx_fp64.json").write_text(json.dumps(rec))


def test_traffic_record_used_only_while_its_sources_match(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    _record(tmp_path, {"k.hip": digest})
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # (FETCH x 2 + WRITE x 1) KiB per dispatch, in bytes
    assert bench.measured_traffic("pair_plane", "CX", "fp64") == (1000.0 * 2 + 500.0) * 1024
    assert bench.measured_traffic("pair_xpass", "CX", "fp64") is None
    assert bench.measured_traffic("pair_plane", "CY", "fp64") is None
    src.write_text("kernel source, changed\n")
    assert bench.measured_traffic("pair_plane", "CX", "fp64") is None
    os.remove(src)
    assert bench.measured_traffic("pair_plane", "CX", "fp64") is None


def test_pair_work_counts_the_occupied_columns_of_the_z_pass():
    # a 60 x 60 x 160 box and an eps "sphere" of three (x, y) columns
    geps = np.array([[0, 0, 0], [0, 0, 1], [0, 0, -1], [1, 0, 0], [0, -2, 5]])
    d = {"box": (60, 60, 160), "nspinor": 2, "nv": 3, "nc": 5, "geps": geps}
    w = bench.pair_work(d)
    f = lambda n: 5.0 * n * np.log2(n)  # noqa: E731
    assert np.isclose(w["pair_xpass"], 15 * f(160) * 3)
    e0 = 2 * 1 + 1  # kept x frequencies: |g_x| <= 1
    plane = (8 * 2 - 2) * 60 * 60 * 160 + f(60) * 60 * 160 + f(60) * e0 * 160
    assert np.isclose(w["pair_plane"], 15 * plane)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
