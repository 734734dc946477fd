"""Host logic of bench.py that needs no GPU: the raster HBM-traffic lookup
from the committed PMC summary (entries per raster kernel, scaling to the
cameras of a launch, null for other kernels or changed raster sources) and
the JSON line's fixed fields."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _recorded_digest():
    with open(os.path.join(ROOT, bench.TRAFFIC_PROFILE)) as fh:
        for line in fh:
            if line.startswith("- sources_sha256: "):
                return line.split(": ", 1)[1].strip().strip("`")
    return None


def test_traffic_summary_has_the_autotuner_kernels_and_scales_per_camera(monkeypatch):
    # the parsing and scaling, independent of whether the summary is current
    monkeypatch.setattr(bench, "raster_source_digest", _recorded_digest)
    for b in (128, 64):
        k = f"gs::k_raster<16, 16, {b}>"
        t512, c = bench.measured_traffic(k, 512)
        assert c == 512 and t512 is not None and t512 > 0
        # per launch, the algorithmic output alone is 512 x 640 x 480 x 20 B
        assert t512 > 512 * 640 * 480 * 20
        t1024, _ = bench.measured_traffic(k, 1024)
        assert t1024 == pytest.approx(2 * t512)
    assert bench.measured_traffic("gs::k_raster<32, 8, 64>", 512) == (None, None)


def test_traffic_is_null_when_the_raster_sources_change(monkeypatch):
    monkeypatch.setattr(bench, "raster_source_digest", lambda: "0" * 64)
    assert bench.measured_traffic("gs::k_raster<16, 16, 128>", 512) == (None, None)


def test_gpus_above_one_exits_with_a_message(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code != 0
    out = capsys.readouterr()
    assert "one GPU" in (out.out + out.err) or "1 GPU" in (out.out + out.err)
