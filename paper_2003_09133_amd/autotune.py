"""Autotuner of the H -> H' kernels: times candidate configurations on the GPU
and writes the winners to the tuning table that liblfbp.so reads at start-up
(paper_2003_09133_amd/lfbp_tune.txt, or $LFBP_TUNE_TABLE).

    python -m paper_2003_09133_amd.autotune [--workloads microscope,camera,camera-f16,batched]
                                            [--out PATH] [--reps N]

A table entry is keyed by (batched, element size, W = ny*nz, nx); shapes with
the same key share the kernel's work decomposition, so one timing serves all
of them.  Inputs are random payloads (the kernels' cost does not depend on the
values).  Only the library's C ABI is called; the choice a run makes is
printed as one JSON line per workload.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "lfbp_tune.txt")
FIELDS = ("variant", "block_threads", "rows_in_flight", "tile_bytes", "vec_per_thread", "nontemporal",
          "persistent", "grid")


def candidates(batched: bool):
    out = []
    for thr, vec, nt in itertools.product((128, 256, 512), (2, 4, 8), (1, 2)):
        out.append({"variant": 3, "block_threads": thr, "vec_per_thread": vec, "nontemporal": nt, "persistent": 2})
    for thr, vec in itertools.product((256, 512), (2, 4)):
        out.append({"variant": 3, "block_threads": thr, "vec_per_thread": vec, "nontemporal": 1, "persistent": 1})
    for thr, rows, tile in itertools.product((256, 512), (1, 2), (8192, 16384, 32768)):
        out.append({"variant": 2, "block_threads": thr, "rows_in_flight": rows, "tile_bytes": tile,
                    "nontemporal": 1, "persistent": 2})
    return out


def _time(fn, torch, reps: int, inner: int = 5) -> float:
    """Median over reps of the mean time of `inner` back-to-back calls (s)."""
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(inner):
            fn()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b) / 1e3 / inner)
    return statistics.median(times)


def full_config(lf, shape, dtype, cfg):
    d = lf.default_config(shape, dtype)
    d.update(cfg)
    d["grid"] = 0
    return d


def read_table(path):
    entries = {}
    if os.path.exists(path):
        with open(path) as fh:
            for line in fh:
                line = line.split("#", 1)[0].split()
                if len(line) == 12:
                    entries[tuple(int(v) for v in line[:4])] = [int(v) for v in line[4:]]
    return entries


def write_table(path, entries, notes):
    with open(path + ".tmp", "w") as fh:
        fh.write("# Tuning table of liblfbp.so, written by paper_2003_09133_amd/autotune.py.\n")
        fh.write("# batched esize W nx | variant threads rows_in_flight tile_bytes vec_per_thread "
                 "nontemporal persistent grid\n")
        for n in notes:
            fh.write(f"# {n}\n")
        for key in sorted(entries):
            fh.write(" ".join(str(v) for v in (*key, *entries[key])) + "\n")
    os.replace(path + ".tmp", path)


def tune_plain(lf, torch, lfsynth, name, reps):
    wname, dt = {"microscope": ("MICROSCOPE", torch.float32), "camera": ("CAMERA", torch.float32),
                 "camera-f16": ("CAMERA", torch.float16)}[name]
    w = getattr(lfsynth, wname)
    H = torch.empty(w.shape, dtype=dt, device="cuda")
    H.view(torch.int32 if dt == torch.float32 else torch.int16).random_(0, 1 << 15)
    Ht = torch.empty_like(H)
    nbytes = 2 * H.numel() * H.element_size()
    results = []
    for cfg in candidates(False):
        t = _time(lambda: lf.compute_Ht_into(H, Ht, config=cfg), torch, reps)
        results.append((nbytes / t / 1e9, cfg))
    results.sort(key=lambda r: -r[0])
    best_gbs, best = results[0]
    esize = H.element_size()
    key = (0, esize, w.shape[3] * w.shape[4], w.shape[2])
    full = full_config(lf, w.shape, dt, best)
    return key, [full[f] for f in FIELDS], {"workload": name, "best_gbs": round(best_gbs, 1), "config": full,
                                            "runner_up": [(round(g, 1), c) for g, c in results[1:4]]}


def tune_batched(lf, torch, lfsynth, reps):
    Hs = []
    for w in lfsynth.BATCHED_SETS:
        h = torch.empty(w.shape, dtype=torch.float32, device="cuda")
        h.view(torch.int32).random_(0, 1 << 15)
        Hs.append(h)
    outs = [torch.empty_like(h) for h in Hs]
    nbytes = sum(2 * h.numel() * 4 for h in Hs)
    results = []
    for cfg in candidates(True):
        t = _time(lambda: lf.compute_Ht_batched(Hs, outs, config=cfg), torch, max(3, reps // 2), inner=2)
        results.append((nbytes / t / 1e9, cfg))
    lf.release_plans()
    results.sort(key=lambda r: -r[0])
    best_gbs, best = results[0]
    big = max(lfsynth.BATCHED_SETS, key=lambda w: w.elements)
    key = (1, 4, big.shape[3] * big.shape[4], big.shape[2])
    full = full_config(lf, big.shape, torch.float32, best)
    return key, [full[f] for f in FIELDS], {"workload": "batched", "best_gbs": round(best_gbs, 1), "config": full,
                                            "runner_up": [(round(g, 1), c) for g, c in results[1:4]]}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workloads", default="microscope,camera,camera-f16,batched")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--reps", type=int, default=7)
    args = ap.parse_args(argv)
    # Tune against the built-in defaults, not an older table.
    os.environ["LFBP_TUNE_TABLE"] = os.path.join(HERE, "_no_table_")
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    import lfsynth
    import paper_2003_09133_amd as lf

    entries = read_table(args.out)
    notes = []
    for name in args.workloads.split(","):
        if name == "batched":
            key, vals, info = tune_batched(lf, torch, lfsynth, args.reps)
        else:
            key, vals, info = tune_plain(lf, torch, lfsynth, name, args.reps)
        entries[key] = vals
        notes.append(f"{info['workload']}: {info['best_gbs']} GB/s on {torch.cuda.get_device_name(0)}")
        print(json.dumps(info), flush=True)
    write_table(args.out, entries, notes)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
