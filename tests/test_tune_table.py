"""The tuning table reader of liblfbp.so (csrc/lfbp_tune.cpp), on the CPU:
entries keyed by (batched, element size, W = ny*nz, nx) replace the built-in
kernel choice; comments, malformed lines and entries with invalid fields are
skipped.  Each case runs in a fresh process, since the library reads the table
once per process (from $LFBP_TUNE_TABLE here)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = """
import json, sys
sys.path.insert(0, {root!r})
import torch
import paper_2003_09133_amd as lf
print(json.dumps([lf.default_config(s, torch.float32) for s in {shapes!r}]))
"""


def configs_with_table(table: str, shapes, tmp_path):
    path = tmp_path / "tune.txt"
    path.write_text(table)
    env = dict(os.environ, LFBP_TUNE_TABLE=str(path))
    r = subprocess.run([sys.executable, "-c", PROBE.format(root=ROOT, shapes=[list(s) for s in shapes])],
                       capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_entries_replace_the_default_and_bad_lines_are_skipped(tmp_path):
    micro = (165, 165, 15, 15, 21)           # W = 315, nx = 15
    other = (45, 45, 9, 9, 7)                # W = 63, nx = 9
    third = (21, 21, 7, 7, 5)                # W = 35, nx = 7
    table = "\n".join([
        "# batched esize W nx variant threads rows tile vec nt persistent grid",
        "0 4 315 15 2 128 1 8192 2 2 2 0   # a staged choice for the microscope key",
        "0 4 63 9 3 100 2 16384 4 1 2 0    # 100 threads: invalid, skipped",
        "0 4 35 7 3 256",                      # malformed, skipped
        "1 4 315 15 1 64 2 0 2 1 1 0       # batched key: not used by plain calls",
    ]) + "\n"
    got = configs_with_table(table, [micro, other, third], tmp_path)
    assert {k: got[0][k] for k in ("variant", "block_threads", "rows_in_flight", "tile_bytes", "nontemporal")} == \
        {"variant": 2, "block_threads": 128, "rows_in_flight": 1, "tile_bytes": 8192, "nontemporal": 2}
    default = configs_with_table("", [other, third], tmp_path)
    assert got[1] == default[0] and got[2] == default[1]
