"""The tuning table reader of liblfbp.so (csrc/lfbp_tune.cpp), on the CPU:
class entries keyed by (batched, element size, row class =
floor(log2(ny*nz*esize))) replace the built-in kernel choice for every shape
of their class, a shape whose class has no entry takes the nearest class's
entry, a shape entry serves its exact shape before any class entry, and
comments, malformed lines and entries with invalid fields are skipped.  Each case runs
in a fresh process, since the library reads the table once per process (from
$LFBP_TUNE_TABLE here)."""
import json
import math
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = """
import json, sys
sys.path.insert(0, {root!r})
import torch
import paper_2003_09133_amd as lf
dt = {{2: torch.float16, 4: torch.float32}}
print(json.dumps([lf.default_config(s, dt[e]) for s, e in {cases!r}]))
"""
FIELDS = ("variant", "block_threads", "rows_in_flight", "tile_bytes", "vec_per_thread", "nontemporal",
          "persistent", "waves_per_eu", "schedule")


def row_class(shape, esize):
    return int(math.floor(math.log2(shape[3] * shape[4] * esize)))


def configs_with_table(table: str, cases, tmp_path):
    path = tmp_path / "tune.txt"
    path.write_text(table)
    env = dict(os.environ, LFBP_TUNE_TABLE=str(path))
    r = subprocess.run([sys.executable, "-c", PROBE.format(root=ROOT, cases=[(list(s), e) for s, e in cases])],
                       capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr
    return [{k: c[k] for k in FIELDS} for c in json.loads(r.stdout.strip().splitlines()[-1])]


def entry(batched, esize, cls, variant, threads, rows, tile, vec, nt, persistent, waves, schedule):
    return (f"class {batched} {esize} {cls} {variant} {threads} {rows} {tile} {vec} {nt} {persistent} 0 "
            f"{waves} {schedule}")


def shape_entry(batched, esize, shape, variant, threads, rows, tile, vec, nt, persistent, waves, schedule):
    return (f"shape {batched} {esize} {' '.join(map(str, shape))} {variant} {threads} {rows} {tile} {vec} {nt} "
            f"{persistent} 0 {waves} {schedule}")


def as_cfg(line):
    v = line.split()
    v = [int(x) for x in v[4:]] if v[0] == "class" else [int(x) for x in v[8:]]
    return dict(zip(FIELDS, v[0:7] + v[8:10]))


def test_class_entries_replace_the_default_and_bad_lines_are_skipped(tmp_path):
    micro = (165, 165, 15, 15, 21)           # row 1260 B: class 10
    same_class = (45, 45, 9, 9, 31)          # row 1116 B: class 10, another shape
    other = (45, 45, 9, 9, 7)                # row 252 B: class 7
    assert row_class(micro, 4) == row_class(same_class, 4) == 10 and row_class(other, 4) == 7
    e10 = entry(0, 4, 10, 2, 128, 1, 8192, 2, 2, 2, 6, 2)
    table = "\n".join([
        "# batched esize class variant threads rows tile vec nt persistent grid waves schedule",
        e10 + "   # a staged choice for class 10",
        entry(0, 4, 7, 3, 100, 2, 16384, 4, 1, 2, 8, 1) + "   # 100 threads: invalid, skipped",
        entry(0, 4, 7, 3, 256, 2, 16384, 4, 1, 2, 9, 1) + "   # 9 waves per SIMD: invalid, skipped",
        "class 0 4 7 3 256 2 16384 4 1 2 0",                        # malformed (too short), skipped
        "0 4 315 15 3 256 2 16384 4 1 2 0",                         # no entry kind, skipped
        "class 0 4 7 3 256 2 16384 4 1 2 0 8 1 5",                  # a field too many, skipped
        "shape 0 4 45 45 9 9 3 256 2 16384 4 1 2 0 8 1",            # shape with four dimensions, skipped
        entry(1, 4, 7, 1, 64, 2, 0, 2, 1, 1, 8, 1) + "   # batched: not used by plain calls",
    ]) + "\n"
    got = configs_with_table(table, [(micro, 4), (same_class, 4), (other, 4)], tmp_path)
    assert got[0] == as_cfg(e10) and got[1] == as_cfg(e10)
    # class 7 has no valid plain entry: the nearest class (10) serves it
    assert got[2] == as_cfg(e10)
    default = configs_with_table("", [(other, 4)], tmp_path)
    assert default[0] != as_cfg(e10)


def test_nearest_class_and_element_size(tmp_path):
    small = (45, 45, 9, 9, 7)                # f32 row 252 B: class 7
    mid = (165, 165, 15, 15, 21)             # f32 class 10, f16 (630 B) class 9
    big = (21, 21, 3, 3, 2000)               # f32 row 24000 B: class 14
    e7 = entry(0, 4, 7, 3, 128, 2, 16384, 2, 2, 2, 8, 1)
    e11 = entry(0, 4, 11, 3, 512, 2, 16384, 4, 1, 2, 4, 2)
    e9h = entry(0, 2, 9, 2, 256, 2, 32768, 4, 2, 2, 8, 1)
    table = "\n".join([e7, e11, e9h]) + "\n"
    got = configs_with_table(table, [(small, 4), (mid, 4), (big, 4), (mid, 2), (small, 2)], tmp_path)
    assert got[0] == as_cfg(e7)               # its own class
    assert got[1] == as_cfg(e11)              # class 10: 11 is one step away, 7 three (and 9 is f16)
    assert got[2] == as_cfg(e11)              # class 14: nearest is 11
    assert got[3] == as_cfg(e9h)              # f16 class 9: its own class and element size
    # f16 class 6: f32 class 7 (one step, other size: 3) beats f16 class 9 (three steps: 6)
    assert row_class(small, 2) == 6 and got[4] == as_cfg(e7)


def test_batched_entries_serve_batched_calls_only(tmp_path):
    """The plain default is unchanged by a batched entry, and a plain entry
    does not become a batched call's configuration (checked through
    default_config, which reports the plain choice)."""
    shape = (165, 165, 15, 15, 21)
    eb = entry(1, 4, 10, 3, 512, 2, 16384, 8, 1, 2, 8, 2)
    got = configs_with_table(eb + "\n", [(shape, 4)], tmp_path)
    default = configs_with_table("", [(shape, 4)], tmp_path)
    assert got == default


def test_shape_entries_come_before_class_entries(tmp_path):
    camera = (345, 345, 15, 15, 51)           # f32 class 11
    near = (345, 345, 15, 15, 49)             # same class, not the same shape
    e11 = entry(0, 4, 11, 3, 256, 2, 16384, 2, 1, 2, 8, 1)
    ecam = shape_entry(0, 4, camera, 3, 128, 2, 16384, 4, 2, 2, 6, 1)
    ecam16 = shape_entry(0, 2, camera, 2, 512, 1, 32768, 4, 2, 2, 8, 2)
    ebat = shape_entry(1, 4, camera, 3, 512, 2, 16384, 8, 1, 2, 8, 2)
    table = "\n".join([e11, ecam, ecam16, ebat]) + "\n"
    got = configs_with_table(table, [(camera, 4), (near, 4), (camera, 2)], tmp_path)
    assert got[0] == as_cfg(ecam)             # the exact shape, f32
    assert got[1] == as_cfg(e11)              # another shape of class 11: the class entry
    assert got[2] == as_cfg(ecam16)           # the exact shape, f16 (the batched shape entry is not used)


def test_partial_retune_keeps_other_entries_and_notes(tmp_path):
    """The autotuner's table bookkeeping (no GPU): a run over a subset keeps the
    other entries, keeps the batched entry only when it does not re-tune it,
    and replaces the note of each re-tuned subject in place."""
    sys.path.insert(0, ROOT)
    from paper_2003_09133_amd import autotune as at
    path = str(tmp_path / "tune.txt")
    cfg = [3, 256, 2, 16384, 4, 1, 2, 0, 8, 1]
    entries = {("class", 0, 4, 10): cfg, ("class", 0, 2, 9): cfg, ("shape", 1, 4, 399, 399, 19, 19, 39): cfg}
    notes = ["camera [345, 345, 15, 15, 51]: 6072.4 GB/s", "f32 class 10: 5908.2 GB/s", "batched: 5980.8 GB/s"]
    at.write_table(path, entries, notes)
    assert at.read_table(path) == entries
    assert at.read_notes(path) == notes
    assert at.kept_entries(at.read_table(path), retune_batched=False) == entries
    assert ("shape", 1, 4, 399, 399, 19, 19, 39) not in at.kept_entries(at.read_table(path), retune_batched=True)
    merged = at.merge_notes(notes, ["f32 class 10: 5950.0 GB/s", "f16 class 12: 5800.0 GB/s"])
    assert merged == ["camera [345, 345, 15, 15, 51]: 6072.4 GB/s", "f32 class 10: 5950.0 GB/s",
                      "batched: 5980.8 GB/s", "f16 class 12: 5800.0 GB/s"]
    assert at.merge_notes([], ["a: 1"]) == ["a: 1"] and at.merge_notes(["a: 1"], []) == ["a: 1"]
