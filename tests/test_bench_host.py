"""Host-side pieces of bench.py (no GPU): the counter-summary lookup that fills
the roofline's `traffic` field, and the algorithmic byte counts."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def write_summary(path, kernel, sha, hbm):
    path.write_text(f"""# a comment line: with colons
kernel: {kernel}
k_vcycle.hip sha256[:16]: {sha}
fetch_bytes_per_launch: 1
write_bytes_per_launch: 2
hbm_bytes_per_launch: {hbm}
""")


def test_traffic_summary_is_read_for_the_current_source(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    write_summary(tmp_path / "k_vc_post_w_fp64_traffic.txt", "k_vc_post", bench.kernel_source_hash(), 12345)
    assert bench.measured_traffic("k_vc_post", "w", "fp64") == 12345.0
    # taken on another source: not used
    write_summary(tmp_path / "k_vc_post_w_fp32_traffic.txt", "k_vc_post", "0000000000000000", 7)
    assert bench.measured_traffic("k_vc_post", "w", "fp32") is None
    assert bench.measured_traffic("k_vc_post", "missing", "fp64") is None


def test_committed_summaries_parse():
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if name.endswith("_traffic.txt"):
            kv = dict(line.rsplit(":", 1) for line in open(os.path.join(ROOT, "profiles", name))
                      if ":" in line and not line.startswith("#"))
            kv = {k.strip(): v.strip() for k, v in kv.items()}
            assert kv["kernel"] == "k_vc_post" and len(kv["k_vcycle.hip sha256[:16]"]) == 16
            assert float(kv["hbm_bytes_per_launch"]) > 0
