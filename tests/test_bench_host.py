"""Host-side checks of bench.py (no GPU): the one-GPU contract, the operation
counts behind the `roofline` objects, and the reading of the committed
profile summaries (kept only when taken on the current kernel sources)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_operation_counts():
    b = _bench()
    # march: GL3 integral with scale (102), 4 projections (44), Kahan (4), exit
    # coordinates (6) in FP32; 13 FP64 operations of the walk
    assert b.FLOPS_PER_CROSSING == {"fp32": 156, "fp64": 13}
    # adjoint scatter: per node 6 + 6 + 17 + 8, the coordinate differences (3) and
    # the retiring face's 4 x 6 products and sums (48)
    assert b.ADJ_FLOPS_PER_CROSSING == {"fp32": 162, "fp64": 13}
    assert b.BYTES_PER_VERTEX == {"fp32": 28, "fp64": 52}


def test_profile_figures_follow_the_source_hash(tmp_path):
    b = _bench()
    src = b.source_hash(b.MARCH_SOURCES)
    good = tmp_path / "good.md"
    good.write_text(f"# x\n\nmarch_source_sha256_16: {src}\nhbm_bytes_per_launch: 1.5e+08\n")
    stale = tmp_path / "stale.md"
    stale.write_text("march_source_sha256_16: 0123456789abcdef\nmarch_l2_hit_frac: 0.5\n")
    got = b.profile_figures((str(good), str(stale)))
    assert got == {"hbm_bytes_per_launch": 1.5e8}
    assert b.profile_figures((str(tmp_path / "missing.md"),)) == {}
    # the adjoint summary is keyed to the adjoint sources, not the march's
    adj = tmp_path / "adj.md"
    adj.write_text(f"adjoint_source_sha256_16: {src}\nscatter_write_bytes_per_launch: 2e9\n")
    assert b.source_hash(b.ADJOINT_SOURCES) != src
    assert b.profile_figures((str(adj),), b.ADJOINT_SOURCES, "adjoint_source_sha256_16") == {}
    adj.write_text(f"adjoint_source_sha256_16: {b.source_hash(b.ADJOINT_SOURCES)}\n"
                   "scatter_write_bytes_per_launch: 2e9\n")
    assert b.profile_figures((str(adj),), b.ADJOINT_SOURCES, "adjoint_source_sha256_16") == \
        {"scatter_write_bytes_per_launch": 2e9}


def test_committed_summaries_carry_the_lines_bench_reads():
    b = _bench()
    for path, tag, keys in (
            (b.TRAFFIC_FILE, "march_source_sha256_16",
             ("hbm_bytes_per_launch", "tensor_hbm_bytes_per_build")),
            (b.COUNTERS_FILE, "march_source_sha256_16",
             ("march_valu_insts_per_crossing", "march_l2_hit_frac", "march_valu_busy_frac")),
            (b.WAVE_FILE, "march_source_sha256_16",
             ("march_hw_fp32_flops_per_crossing", "march_lane_utilisation")),
            (b.ADJOINT_FILE, "adjoint_source_sha256_16",
             ("scatter_write_bytes_per_launch", "scatter_valu_insts_per_wave_crossing"))):
        txt = open(path).read()
        assert tag + ":" in txt, path
        for k in keys:
            assert k + ":" in txt, (path, k)
