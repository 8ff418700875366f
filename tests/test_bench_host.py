"""Host logic of the benchmark's measurement (no GPU): the kernel-source hash
that gates stored HBM counters, the reading of a committed traffic summary,
the CSR byte convention and the choice of the dominant kernel."""
import os
import shutil
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _copy_sources(dst):
    for f in bench.KERNEL_SOURCES:
        os.makedirs(os.path.join(dst, os.path.dirname(f)), exist_ok=True)
        shutil.copy(os.path.join(ROOT, f), os.path.join(dst, f))


def test_source_hash_ignores_comments_and_blank_lines_only(tmp_path, monkeypatch):
    _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    assert h0 == bench.kernel_source_hash()
    src = os.path.join(tmp_path, bench.KERNEL_SOURCES[0])
    text = open(src).read()
    with open(src, "w") as f:
        f.write("// a comment line\n\n" + text.replace("\n", "  // trailing comment\n", 3))
    assert bench.kernel_source_hash() == h0
    with open(src, "w") as f:
        f.write(text + "\nstatic int an_added_line = 0;\n")
    assert bench.kernel_source_hash() != h0


def test_traffic_is_read_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_traffic("abc", "k_demo") is None  # no summary
    os.makedirs(tmp_path / "profiles")
    (tmp_path / "profiles" / "k_demo_traffic.txt").write_text(
        "# rocprofv3 HBM counters\ncommand (fetch): cd /tmp && rocprofv3 --pmc FETCH_SIZE -- python3 x.py\n"
        "kernel_source_sha256: abc\nhbm_bytes_per_launch: 3346551345\n")
    assert bench.read_traffic("abc", "k_demo") == 3346551345.0
    assert bench.read_traffic("abd", "k_demo") is None
    (tmp_path / "profiles" / "k_demo_traffic.txt").write_text("kernel_source_sha256: abc\n")
    assert bench.read_traffic("abc", "k_demo") is None  # no byte count


def test_committed_headline_summaries_share_one_source_hash():
    # the trace, traffic and counter summaries of the headline kernel were
    # taken on the same sources
    stem = os.path.join(ROOT, "profiles", "k_cwin2048_fp64_hex27_16M_rcm")
    hashes = set()
    for part in ("ktrace", "traffic", "counters"):
        with open(f"{stem}_{part}.txt") as f:
            hashes |= {ln.split(":", 1)[1].strip() for ln in f if ln.startswith("kernel_source_sha256:")}
    assert len(hashes) == 1


def test_csr_byte_convention():
    # each stored entry: its value and a 4-byte column index; row_ptr; x read
    # once and y written once
    n_rows, n_cols, nnz = 16003008, 16003008, 270148760
    assert bench.alg_bytes(n_rows, n_cols, nnz, 8, 8, 8) == 3561845284
    assert bench.alg_bytes(3, 5, 7, 4, 2, 8) == 7 * 8 + 4 * 4 + 2 * 5 + 8 * 3
    assert bench.alg_bytes(0, 0, 0, 8, 8, 8) == 4


@pytest.mark.parametrize("win,tiles,expect", [(132330, 132628, "k_cwin2048"), (10, 132628, "k_stream2048")])
def test_dominant_kernel_follows_the_plan(win, tiles, expect):
    name, stem = bench.dominant_kernel({"n_window_tiles": win, "n_tiles": tiles, "tile_nnz": 2048})
    assert stem.startswith(expect) and name.startswith(expect[:-4] + "<double")


def test_serving_child_is_ended_when_it_stops_printing(monkeypatch):
    monkeypatch.setattr(bench, "SERVE_STALL_S", 2)
    quiet = [sys.executable, "-c", "import sys, time; print('step', file=sys.stderr, flush=True); time.sleep(60)"]
    r = bench.serving_in_child(None, cmd=quiet)
    assert r == {"failed": "no progress for 2 s"}
    talk = [sys.executable, "-c", "import sys, time\n"
            "for i in range(4):\n    print('step', i, file=sys.stderr, flush=True); time.sleep(0.5)\n"
            "print('{\"preloaded\": {\"p50_ms\": 1.0}}', flush=True)"]
    assert bench.serving_in_child(None, cmd=talk) == {"preloaded": {"p50_ms": 1.0}}
    failing = [sys.executable, "-c", "raise SystemExit(3)"]
    assert bench.serving_in_child(None, cmd=failing) == {"failed": "child exit status 3"}
