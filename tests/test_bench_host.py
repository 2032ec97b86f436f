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


def _counter_csv(path, rows):
    import csv
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_traffic_summary_counts_32_byte_units(tmp_path):
    """32 x the request counts, averaged over working dispatches only (the
    ones that return at once on the done flag are left out), the four-step
    update weighted 1:3, and the copy's reading reported as the check."""
    import json

    import bench
    R, W = bench.DRAM_READ, bench.DRAM_WRITE
    mib = 1
    copy_units = mib * (1 << 20) // 32
    _counter_csv(tmp_path / "copy.csv", [(i, "copy", c, copy_units) for i in range(20)
                                         for c in (R, W)])
    rows = []
    did = 0
    for reads, writes in [(1000, 500), (1200, 700), (3, 1)]:  # the last one returned at once
        rows += [(did, "void fs::k_dir_spmv_zm<0, false>(int, int)", R, reads),
                 (did, "void fs::k_dir_spmv_zm<0, false>(int, int)", W, writes)]
        did += 1
    for name, reads in [("void fs::k_update4<4, true, false>(int)", 4000),
                        ("void fs::k_update4<4, false, false>(int)", 2000)]:
        rows += [(did, name, R, reads), (did, name, W, 0)]
        did += 1
    _counter_csv(tmp_path / "run.csv", rows)
    out = tmp_path / "profiles"
    out.mkdir()
    written = bench.summarize_traffic(str(tmp_path / "run.csv"), str(tmp_path / "copy.csv"),
                                      "jacobi", 16, ["cmd"], str(out), copy_mib=mib)
    recs = {}
    for p in written:
        line = [l for l in open(p).read().splitlines() if l.startswith("bench-traffic:")][0]
        rec = json.loads(line.split(":", 1)[1])
        recs[rec["kind"]] = rec
    spmv = recs["pcg_dir_spmv"]
    assert spmv["read_bytes"] == 32 * 1100 and spmv["write_bytes"] == 32 * 600
    assert spmv["copy_check"] == [1.0, 1.0]
    assert spmv["algorithmic_bytes"] == 17 * 16 ** 3
    upd = recs["pcg_update"]
    assert upd["read_bytes"] == int(32 * (0.25 * 4000 + 0.75 * 2000))
