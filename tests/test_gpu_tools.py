"""The autotuner and the benchmark as a user runs them, on the GPU, each in a
process of its own: the autotuner writes a tuning table whose entry the
library then uses, and bench.py prints one JSON line with every field of its
contract."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.gpu


def run(args, env=None, timeout=240):
    r = subprocess.run([sys.executable, *args], cwd=ROOT, capture_output=True, text=True, timeout=timeout,
                       env=dict(os.environ, **(env or {})))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    return r.stdout


def test_autotuner_writes_a_table_the_library_uses(tmp_path):
    """One row class tuned into a fresh table: a shape of that class that the
    tuner never ran (and a shape of another class, through the nearest-class
    rule) then runs the tuned configuration."""
    table = tmp_path / "tune.txt"
    out = run(["-m", "paper_2003_09133_amd.autotune", "--classes", "f32:10", "--shapes", "", "--no-batched",
               "--reps", "1", "--out", str(table)])
    report = json.loads([l for l in out.splitlines() if l.startswith("{")][-1])
    assert report["class"] == [4, 10] and report["best_gbs"] > 0 and report["default_gbs"] > 0
    rows = [l.split() for l in table.read_text().splitlines() if l.strip() and not l.startswith("#")]
    assert len(rows) == 1 and len(rows[0]) == 14
    key, cfg = rows[0][:4], [int(v) for v in rows[0][4:]]
    assert key == ["class", "0", "4", "10"]                   # plain, float32, rows of 1024..2047 bytes
    unseen = [(45, 45, 9, 9, 31), (209, 209, 11, 11, 22)]    # rows of 1116 B (class 10) and 968 B (class 9)
    probe = ("import json, sys; sys.path.insert(0, %r); import torch, paper_2003_09133_amd as lf; "
             "print(json.dumps([lf.default_config(s, torch.float32) for s in %r]))" % (ROOT, unseen))
    used = json.loads(run(["-c", probe], env={"LFBP_TUNE_TABLE": str(table)}).strip().splitlines()[-1])
    fields = ("variant", "block_threads", "rows_in_flight", "tile_bytes", "vec_per_thread", "nontemporal",
              "persistent", "grid", "waves_per_eu", "schedule")
    want = dict(zip(fields, cfg))
    for u in used:
        assert {f: u[f] for f in fields if f != "grid"} == {f: want[f] for f in fields if f != "grid"}


def test_shipped_table_against_builtin_default_on_unseen_shapes():
    """Three PSF shapes that no table entry was tuned on (sets of the 16-set
    table, three row classes), timed with the shipped table's choice and with
    the built-in default: the class entries serve them, and the gap is
    printed (the tuned choice is not allowed to be much slower)."""
    spec = "165,165,15,15,35;209,209,11,11,22;285,285,19,19,20"
    tuned = json.loads(run(["-m", "paper_2003_09133_amd.autotune", "--time-shapes", spec, "--reps", "5"]
                           ).strip().splitlines()[-1])
    default = json.loads(run(["-m", "paper_2003_09133_amd.autotune", "--time-shapes", spec, "--reps", "5"],
                             env={"LFBP_TUNE_TABLE": os.path.join(ROOT, "_no_table_")}).strip().splitlines()[-1])
    for t, d in zip(tuned, default):
        print(f"{t['shape']} class {t['row_class']}: tuned {t['GBs']} GB/s, built-in default {d['GBs']} GB/s "
              f"({t['GBs'] / d['GBs']:.3f}x)")
        assert t["GBs"] > 0.9 * d["GBs"], (t, d)


def test_bench_line_carries_every_field():
    out = run(["bench.py", "--workload", "tiny", "--steps", "3", "--warmup", "1", "--cpu-seconds", "1"])
    lines = [l for l in out.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1 and d["value"] > 0
    assert d["config"]["workload"]
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["unit"] == "GB/s"
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0 and c["sample"]
    dev = d["config"]["device"]
    assert dev["compute_units"] > 0 and dev["arch"].startswith("gfx")


def test_bench_microscope_line_after_a_buffer_between_calls():
    """The microscope line carries the build timed after a 1 GiB buffer is
    written and after it is read between calls, and its output matches the
    oracle bit for bit."""
    out = run(["bench.py", "--workload", "microscope", "--steps", "3", "--warmup", "1", "--cpu-seconds", "1"])
    d = json.loads([l for l in out.splitlines() if l.startswith("{")][-1])
    fl = d["config"]["after_1GiB_buffer"]
    for mode in ("written", "read"):
        assert fl[mode]["GBs_at_median"] > 0 and fl[mode]["step_ms"]["min"] > 0
    assert all(v["mismatches"] == 0 for v in d["config"]["bit_exact_vs_oracle"].values())


def test_default_config_reports_what_a_launch_runs():
    """In a fresh process, the configuration lfbp_default_config reports for a
    shape with rows over 32 KB (whose work decomposition depends on the
    device's LDS size) is the same before and after the first build, grid
    included, and the build with that configuration passed explicitly equals
    the default build bit for bit."""
    probe = ("import json, sys; sys.path.insert(0, %r); import torch, paper_2003_09133_amd as lf\n"
             "shape = (3, 3, 3, 3, 3001)\n"
             "before = lf.default_config(shape, torch.float32)\n"
             "H = torch.rand(shape, device='cuda')\n"
             "ref = lf.compute_Ht(H)\n"
             "after = lf.default_config(shape, torch.float32)\n"
             "got = lf.compute_Ht(H, config=after)\n"
             "print(json.dumps([before, after, bool(torch.equal(ref.view(torch.int32), got.view(torch.int32)))]))"
             % ROOT)
    before, after, same = json.loads(run(["-c", probe]).strip().splitlines()[-1])
    assert 3 * 3001 * 4 > 32 * 1024
    assert before == after, (before, after)
    assert same
