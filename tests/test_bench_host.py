"""Host-side parts of the benchmark: the one-GPU guard and the counter
records that supply roofline.traffic (valid only while the kernel sources
hash to the recorded value)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_traffic_record_requires_matching_sources(tmp_path):
    h = bench.sources_hash(bench.NET_SOURCES)
    rec = tmp_path / "rec.md"
    rec.write_text(f"# k\n\n- hbm_bytes_per_launch: `12345`\n- sources_sha256: `{h}`\n")
    val, src = bench.recorded_traffic(str(rec), bench.NET_SOURCES)
    assert val == 12345.0
    rec.write_text("- hbm_bytes_per_launch: `12345`\n- sources_sha256: `0000000000000000`\n")
    val, why = bench.recorded_traffic(str(rec), bench.NET_SOURCES)
    assert val is None and "changed" in why
    val, why = bench.recorded_traffic(str(tmp_path / "missing.md"), bench.NET_SOURCES)
    assert val is None


@pytest.mark.parametrize("kernel", sorted(bench.TRAFFIC_RECORDS))
def test_committed_records_parse(kernel):
    path = bench.TRAFFIC_RECORDS[kernel]
    if not os.path.exists(path):
        pytest.skip("no record for this kernel")
    text = open(path).read()
    assert "hbm_bytes_per_launch" in text and "sources_sha256" in text and "rocprofv3" in text
