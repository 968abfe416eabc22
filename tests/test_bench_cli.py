"""The benchmark's command-line contract that needs no GPU: one GPU only."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_traffic_summary_lookup(tmp_path):
    """The roofline's traffic figure is read only when the summary was taken
    on the same kernel sources and launch shape."""
    sys.path.insert(0, ROOT)
    import bench
    src = ["kernels_plain.hip", "stencil_plain.h", "reduce.h", "internal.h"]
    h = bench.kernel_source_hash(src)
    assert len(h) == 16
    assert bench.read_traffic("step_plain", "pulsed_256x256x200", "0" * 16, "tile_x 0 tile_y 8 z_chunk 0") is None
    assert bench.read_traffic("step_plain", "no_such_workload", h, "tile_x 0 tile_y 8 z_chunk 0") is None


def test_source_hash_ignores_comments(tmp_path):
    """A counter summary survives an edit of a comment, not of code."""
    sys.path.insert(0, ROOT)
    import bench
    code = "__global__ void k(double* x) {  // one store\n  x[0] = 1.0; /* the value */\n}\n"
    (tmp_path / "k.hip").write_text(code)
    h = bench.kernel_source_hash(["k.hip"], str(tmp_path))
    (tmp_path / "k.hip").write_text("// a kernel\n" + code.replace("one store", "a store") + "\n\n")
    assert bench.kernel_source_hash(["k.hip"], str(tmp_path)) == h
    (tmp_path / "k.hip").write_text(code.replace("1.0", "2.0"))
    assert bench.kernel_source_hash(["k.hip"], str(tmp_path)) != h


def test_a_failing_extra_section_is_reported_in_the_line(capsys):
    """An extra section that raises becomes {"error": ...} in its field (the
    headline measured before it is still printed); one that works returns
    its dict."""
    sys.path.insert(0, ROOT)
    import bench

    def broken():
        raise RuntimeError("it_solve_batch: stand-in failure")
    assert bench.run_section("sweep", lambda: {"seconds": 1.0}) == {"seconds": 1.0}
    out = bench.run_section("sweep", broken)
    assert "stand-in failure" in out["error"]
    assert "sweep: failed" in capsys.readouterr().err
    json.dumps(out)
