"""Host logic of the benchmark (no GPU): every committed counter summary
still matches the kernel sources it was taken from, and a multi-GPU request
is refused with a message."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _summaries():
    out = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        kind, precond, n = os.path.basename(path)[:-len("_traffic.md")].rsplit("_", 2)
        out.append((kind, precond, int(n)))
    return out


@pytest.mark.parametrize("kind,precond,n", _summaries())
def test_traffic_summaries_match_current_sources(kind, precond, n):
    import bench
    got = bench.load_traffic(kind, n, precond)
    assert got is not None and got > 0, (
        f"profiles/{kind}_{precond}_{n}_traffic.md no longer matches its kernel sources")


def test_traffic_summary_rejects_a_changed_source(tmp_path, monkeypatch):
    import bench
    kind, precond, n = _summaries()[0]
    src = open(os.path.join(ROOT, "profiles", f"{kind}_{precond}_{n}_traffic.md")).read()
    fake = tmp_path / "profiles"
    fake.mkdir()
    (fake / f"{kind}_{precond}_{n}_traffic.md").write_text(src)
    # the same summary next to a copy of the sources with one byte changed
    import json
    rec = json.loads([l for l in src.splitlines() if l.startswith("bench-traffic:")][0].split(":", 1)[1])
    for rel in rec["sources"]:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_bytes(open(os.path.join(ROOT, rel), "rb").read())
    first = tmp_path / next(iter(rec["sources"]))
    first.write_bytes(first.read_bytes() + b"\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic(kind, n, precond) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
