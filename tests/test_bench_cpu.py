"""Host-side plumbing of bench.py: argument handling, the CPU baseline leg, and the JSON
line that must be printed even when a section fails (no GPU needed)."""
from __future__ import annotations

import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as W  # noqa: E402


def test_driver_flags_parse():
    a = bench.parse_args(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert (a.gpus, a.steps, a.warmup, a.cpu_steps) == (1, 20, 5, 24)


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU only" in capsys.readouterr().err


def test_cpu_baseline_wavelet_shorter_than_sample():
    # the GPU leg ran 5 steps, so the shot's wavelet has 5 samples; the baseline asks for
    # 16 and must build its own wavelet of that length
    shot = W.c0(nt=5)
    assert shot.wavelet.shape == (5,)
    cpu = bench.cpu_baseline(shot, 16)
    assert cpu["kind"] == "oracle" and cpu["unit"] == "Gcell-steps/s"
    assert cpu["value"] > 0 and cpu["cores"] >= 1
    assert cpu["one_core"]["steps"] == 2 and cpu["one_core"]["value"] > 0
    assert "64x64x64" in cpu["sample"] and "first 16 steps" in cpu["sample"]


def test_line_printed_when_sections_fail(monkeypatch, capsys):
    def boom(*a, **k):
        raise RuntimeError("no device here")

    monkeypatch.setattr(bench, "Forward", boom)
    monkeypatch.setattr(bench, "stream_copy_ceiling", boom)
    rc = bench.main(["--steps", "20", "--warmup", "5", "--no-c2", "--no-batch", "--no-grad", "--no-levels",
                     "--no-born", "--no-coarse", "--no-layout-ab", "--cpu-steps", "0"])
    assert rc == 1
    lines = [l for l in capsys.readouterr().out.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    out = json.loads(lines[0])
    assert out["value"] is None and out["roofline"] is None
    assert set(out["errors"]) == {"forward", "stream_copy_gbs"}
    assert "no device here" in out["errors"]["forward"]
    assert out["n_gpus"] == 1 and out["steps"] == 20 and out["warmup"] == 5
    assert out["paper_table6"]["levels"][7]["grid"] == [256, 256, 256]


def test_line_carries_roofline_fields():
    args = bench.parse_args(["--steps", "20", "--warmup", "5"])
    f = dict(gcs=45.0, elapsed=0.0075, times=[0.0075, 0.0076, 0.0074], per={"velocity": 0.17, "stress": 0.2},
             per_kernel={"velocity": dict(avg_ms=0.17, achieved_gbs=5130.0, frac=0.641),
                         "stress": dict(avg_ms=0.2, achieved_gbs=5704.0, frac=0.713)},
             dom="stress", kernel={"variant": "tile", "tile_x": 256, "tile_y": 4, "zchunk": 64},
             bytes_launch=68 * 256 ** 3, events_gbs=5441.0, wall_gbs=5400.0, traffic=None)
    out = bench.build_line(args, {"forward": f, "cpu_baseline": {"value": 0.05}}, {})
    r = out["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-3)
    assert r["whole_step"]["bytes_per_cell"] == 120
    assert out["errors"] is None and out["cpu_baseline"]["value"] == 0.05
    assert out["config"]["hbm_frac_whole_step"] == pytest.approx(5400.0 / 8000.0, rel=1e-3)


def test_paper_table6_rates():
    ctx = bench.paper_context()
    lev7 = ctx["levels"][7]
    # level 7: 256^3 x 17000 steps in 48 min 10 s on the paper's iGPU
    assert lev7["gpu_s"] == 48 * 60 + 10
    assert lev7["gpu_gcs"] == pytest.approx(256 ** 3 * 17000 / 2890 / 1e9, rel=1e-3)


def test_traffic_table_is_keyed_by_layout():
    # the committed counter table holds HBM bytes per configuration and field layout; a
    # configuration it does not hold reports no traffic
    k = {"variant": "tile", "tile_x": 256, "tile_y": 4, "zchunk": 64}
    got = {lay: bench.measured_traffic(dict(k, layout=lay), "stress") for lay in ("separate", "rows", "nope")}
    assert got["nope"] is None
    for lay in ("separate", "rows"):
        assert got[lay] is None or 1.0 <= got[lay] / (68 * 256 ** 3) <= 1.2, (lay, got[lay])
    assert got["separate"] is not None or got["rows"] is not None
