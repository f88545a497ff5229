"""bench.py's contract on the host: more than one GPU is refused before anything runs."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_a_failed_comparison_is_recorded_and_the_line_still_printed(monkeypatch, capsys):
    """The headline line must survive a comparison that raises (host logic only: the
    measurements are stand-ins)."""
    import json
    sys.path.insert(0, ROOT)
    import bench

    class W:
        lattice, name, nx, ny = "D2Q4", "euler2d", 8, 8

    def fake_single(args, torch):
        return {"metric": bench.METRIC, "value": 1.0, "roofline": {}}, W()

    def boom(*a, **k):
        raise RuntimeError("stand-in failure")

    monkeypatch.setattr(bench, "bench_single", fake_single)
    monkeypatch.setattr(bench, "single_run", lambda torch, w, reps, warm_steps: {"mlups": 1.0})
    monkeypatch.setattr(bench, "batch_compare", boom)
    monkeypatch.setattr(bench, "adjoint_compare", lambda *a, **k: {"ratio_to_forward": 4.0})
    monkeypatch.setattr(bench, "riemann_compare", lambda torch: {})
    monkeypatch.setattr(bench, "cpu_baseline", lambda w: {"value": 0.01})
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    bench.main()
    lines = [l for l in capsys.readouterr().out.splitlines() if l.strip()]
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert rec["value"] == 1.0 and rec["c1"] == {"mlups": 1.0}
    assert rec["batch"] == {"error": "RuntimeError: stand-in failure"}
    assert rec["adjoint"]["ratio_to_forward"] == 4.0 and rec["cpu_baseline"]["value"] == 0.01
