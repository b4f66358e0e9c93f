"""bench.py's host side (no GPU): the one-GPU rule, the Table 1 fixture it
reports beside the column-major timings, and its profile readers."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import lfsynth  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_table1_fixture_covers_every_size():
    secs = bench.table1_paper_seconds()
    assert set(secs) == set(lfsynth.TABLE1_SHAPES)
    assert all(s > 0 for s in secs.values())
    assert secs[(181, 95, 55)] == 5.9 and secs[(89, 11, 11)] == 0.1


def test_profile_readers_return_none_or_bytes():
    """Traffic figures come from the committed counter summaries only when
    their recorded source digest matches the current sources."""
    for v in (bench.traffic_from_profile("microscope"), bench.projector_traffic(),
              bench.colmajor_traffic([307, 307, 51, 51, 11]), bench.step_traffic("rl"),
              bench.step_traffic("grad-psf")):
        assert v is None or (isinstance(v, int) and v > 0)
    assert bench.traffic_from_profile("no-such-workload") is None
    assert bench.step_traffic("no-such-workload") is None
    assert bench.colmajor_traffic([3, 3, 3, 3, 3]) is None
