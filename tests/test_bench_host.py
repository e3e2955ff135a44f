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


def test_byte_counts_of_the_timed_kernel_at_128():
    """Level-0 prolongation + postsmoothing of the 128^3 Poisson system:
    the byte model 12 nnz + 32 N + 8 N_c, and the implementation's count
    (row pointers, values and columns, the prolongated iterate, D^{-1}, the
    result, and r read once, from which g = D^{-1} r is formed)."""
    n, nnz, nc = 128 ** 3, 7 * 128 ** 3 - 6 * 128 ** 2, 64 * 64 * 128
    sizes = [(n, nnz), (nc, 7 * nc)]
    assert bench.model_bytes(sizes, 8) == 12 * nnz + 32 * n + 8 * nc == 246284288
    assert bench.kernel_bytes(sizes, 8, "pcg")[0] == 12 * nnz + 4 * (n + 1) + 32 * n
    # the float preconditioner reads g (float) and, for PCG's (r, z), r
    assert bench.kernel_bytes(sizes, 4, "pcg")[0] == 8 * nnz + 4 * (n + 1) + 8 * n + 8 * n + 4 * n + 8 * n
    assert bench.model_bytes(sizes, 4) == 8 * nnz + 32 * n + 8 * nc


def test_host_description():
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and (h["model"] is None or isinstance(h["model"], str))
