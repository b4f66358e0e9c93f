"""Autotuner of the H -> H' kernels: times candidate configurations on the GPU
and writes the winners to the tuning table that liblfbp.so reads at start-up
(paper_2003_09133_amd/lfbp_tune.txt, or $LFBP_TUNE_TABLE).

    python -m paper_2003_09133_amd.autotune [--classes f32:7,...,f16:10] [--shapes camera,...]
                                            [--no-batched] [--out PATH] [--reps N]
    python -m paper_2003_09133_amd.autotune --time-shapes "ns,nt,nx,ny,nz[:f16];..."

The table holds two kinds of entries.  A class entry is keyed by (batched,
element size, row class), the row class of a shape being
floor(log2(ny*nz*esize)): the kernels cut H into units of whole x-rows, so the
size of a row decides the work decomposition; a shape with no entry of its
own takes its class's entry, or the nearest class's.  A shape entry serves
one exact shape: the named PSF workloads (SHAPE_WORKLOADS), and the batched
16-set table (keyed by its largest problem).  Every sweep has two stages:
kernel variant, workgroup size, loads per thread and store kind first, then
occupancy cap (waves per SIMD) and the order in which units meet the XCDs for
the best of those.  Each class is tuned on five or six representative PSF
shapes whose rows span the class (CLASS_SHAPES): a candidate that is more than 2% slower than the built-in
default on any of them is passed over, the others are ranked by the geometric
mean of their rates, and a class whose best candidate does not beat the
default by MIN_GAIN keeps the default.  Every winner's output is compared
bit for bit with the built-in default's before it is written.  The batched
entry is tuned in a child process that reads the freshly written plain
entries (a batch cuts each problem into units of its plain entry's size).
A run over some of the shapes and classes keeps the table's other entries (and
the batched entry under --no-batched) and their notes.
Inputs are random payloads (the kernels' cost does not depend on the values).
Only the library's C ABI is called.  --time-shapes prints, for each shape,
the configuration the library picks and its rate (GB/s), as one JSON line.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import statistics
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "lfbp_tune.txt")
FIELDS = ("variant", "block_threads", "rows_in_flight", "tile_bytes", "vec_per_thread", "nontemporal",
          "persistent", "grid", "waves_per_eu", "schedule")

# Representative PSF shapes (ns, nt, nx, ny, nz) of each (element size, row
# class): odd cells and patches of an odd number of whole lenslets, 0.2 to
# 5.5 GB per array, different cell sizes and depth counts, with rows from the
# low to the high end of the class.  A configuration is
# scored by the geometric mean of its rates over the class's shapes, so that
# the entry serves the whole class rather than one shape.
CLASS_SHAPES = {
    (4, 7): [(497, 497, 7, 7, 7), (405, 405, 9, 9, 6), (693, 693, 11, 11, 5), (385, 385, 7, 7, 9),
             (495, 495, 11, 11, 3)],
    (4, 8): [(405, 405, 9, 9, 11), (735, 735, 7, 7, 12), (253, 253, 11, 11, 9), (165, 165, 15, 15, 8),
             (325, 325, 13, 13, 5), (385, 385, 7, 7, 18)],
    (4, 9): [(275, 275, 11, 11, 20), (525, 525, 15, 15, 10), (245, 245, 7, 7, 30), (165, 165, 15, 15, 15),
             (275, 275, 11, 11, 12), (245, 245, 7, 7, 36)],
    (4, 10): [(165, 165, 15, 15, 21), (171, 171, 19, 19, 25), (297, 297, 11, 11, 30), (135, 135, 15, 15, 30),
              (195, 195, 13, 13, 20), (165, 165, 15, 15, 34)],
    (4, 11): [(345, 345, 15, 15, 51), (225, 225, 15, 15, 45), (209, 209, 11, 11, 60), (135, 135, 15, 15, 40),
              (195, 195, 15, 15, 35), (135, 135, 15, 15, 68)],
    (4, 12): [(171, 171, 19, 19, 80), (135, 135, 15, 15, 100), (99, 99, 11, 11, 120), (75, 75, 15, 15, 90),
              (135, 135, 15, 15, 69), (75, 75, 15, 15, 136)],
    (4, 13): [(105, 105, 15, 15, 200), (57, 57, 19, 19, 150), (77, 77, 11, 11, 300), (45, 45, 15, 15, 250),
              (75, 75, 15, 15, 137), (45, 45, 15, 15, 272)],
    (4, 14): [(45, 45, 15, 15, 300), (57, 57, 19, 19, 300), (31, 31, 31, 31, 200), (75, 75, 15, 15, 400),
              (75, 75, 15, 15, 274), (45, 45, 15, 15, 545)],
}
# float16 rows of a shape are half as long as its float32 rows: the float16
# class c is tuned on the shapes of the float32 class c + 1.
CLASS_SHAPES.update({(2, c): CLASS_SHAPES[(4, c + 1)] for c in range(6, 14)})
# A tuned class entry must beat the built-in default by this factor (geometric
# mean over the class's shapes), and may be at most MAX_LOSS slower than it on
# any one of them; otherwise the class keeps the default.
MIN_GAIN = 1.005
MAX_LOSS = 0.98
# Named PSF workloads tuned for their exact shape: (name, shape, element size).
SHAPE_WORKLOADS = {
    "camera": ((345, 345, 15, 15, 51), 4),
    "camera-f16": ((345, 345, 15, 15, 51), 2),
    "microscope": ((165, 165, 15, 15, 21), 4),
}


def row_class(shape, esize: int) -> int:
    b = shape[3] * shape[4] * esize
    return b.bit_length() - 1


def stage1(batched: bool):
    out = []
    for thr, vec, nt in itertools.product((128, 256, 512), (2, 4, 8), (1, 2)):
        out.append({"variant": 3, "block_threads": thr, "vec_per_thread": vec, "nontemporal": nt, "persistent": 2})
    for thr, vec in itertools.product((256, 512), (2, 4)):
        out.append({"variant": 3, "block_threads": thr, "vec_per_thread": vec, "nontemporal": 2, "persistent": 1})
    if not batched:
        for thr, rows, tile in itertools.product((256, 512), (1, 2), (8192, 16384, 32768)):
            out.append({"variant": 2, "block_threads": thr, "rows_in_flight": rows, "tile_bytes": tile,
                        "nontemporal": 1, "persistent": 2})
    return out


def stage2(best: dict):
    out = []
    for waves, sched in itertools.product((8, 6, 5, 4), (1, 2)):
        c = dict(best)
        c.update({"waves_per_eu": waves, "schedule": sched})
        out.append(c)
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
    """Entries of a table file: {key: config fields}, key = ("class", batched,
    esize, class) or ("shape", batched, esize, ns, nt, nx, ny, nz)."""
    entries = {}
    if os.path.exists(path):
        with open(path) as fh:
            for line in fh:
                f = line.split("#", 1)[0].split()
                if f and f[0] == "class" and len(f) == 14:
                    entries[("class", *(int(v) for v in f[1:4]))] = [int(v) for v in f[4:]]
                elif f and f[0] == "shape" and len(f) == 18:
                    entries[("shape", *(int(v) for v in f[1:8]))] = [int(v) for v in f[8:]]
    return entries


HEADER_LINES = 4   # fixed comment lines at the top of a table file (written by write_table)


def read_notes(path):
    """The note lines of a table file (comments after the fixed header), in order."""
    if not os.path.exists(path):
        return []
    with open(path) as fh:
        comments = [l[1:].strip() for l in fh if l.startswith("#")]
    return comments[HEADER_LINES:]


def merge_notes(old, new):
    """Notes of a partial re-tune: a new note replaces the old note on the same
    subject (the text before its first colon) in place; other old notes stay,
    and new subjects follow them."""
    subject = lambda n: n.split(":", 1)[0]
    fresh = {subject(n): n for n in new}
    out = [fresh.pop(subject(n), n) for n in old]
    return out + [n for n in new if subject(n) in fresh]


def kept_entries(entries, retune_batched):
    """Entries of an existing table that a run keeps before it adds its own:
    every plain entry, and the batched entry unless the run re-tunes it."""
    return {k: v for k, v in entries.items() if k[1] == 0 or not retune_batched}


def write_table(path, entries, notes):
    with open(path + ".tmp", "w") as fh:
        fh.write("# Tuning table of liblfbp.so, written by paper_2003_09133_amd/autotune.py.\n")
        fh.write("# shape batched esize ns nt nx ny nz | config\n")
        fh.write("# class batched esize row_class | config\n")
        fh.write("# config = variant threads rows_in_flight tile_bytes vec_per_thread nontemporal persistent grid "
                 "waves_per_eu schedule\n")
        for n in notes:
            fh.write(f"# {n}\n")
        for key in sorted(entries, key=lambda k: (k[0] != "shape", k[1:])):
            fh.write(" ".join(str(v) for v in (*key, *entries[key])) + "\n")
    os.replace(path + ".tmp", path)


def random_psf(torch, shape, dtype):
    H = torch.empty(shape, dtype=dtype, device="cuda")
    H.view(torch.int32 if dtype == torch.float32 else torch.int16).random_(0, 1 << 15)
    return H


def same_bits(torch, a, b) -> bool:
    it = torch.int32 if a.element_size() == 4 else torch.int16
    return bool(torch.equal(a.view(it), b.view(it)))


def geomean(v):
    p = 1.0
    for x in v:
        p *= x
    return p ** (1.0 / len(v))


def sweep(runs, torch, reps, inner, batched, floor=None):
    """Two-stage sweep over (run(cfg), bytes) pairs, scored by the geometric
    mean of the rates; with `floor` (per-run GB/s), a candidate slower than
    floor on any run is passed over.  Returns (best score in GB/s, best
    config, ranked results as (score, config, per-run GB/s)); the config is
    None when every candidate was passed over."""
    def score(cfg):
        rates = [nb / _time(lambda: run(cfg), torch, reps, inner) / 1e9 for run, nb in runs]
        ok = floor is None or all(r >= f for r, f in zip(rates, floor))
        return (geomean(rates) if ok else 0.0), cfg, [round(r, 1) for r in rates]
    results = [score(cfg) for cfg in stage1(batched)]
    results.sort(key=lambda r: -r[0])
    if results[0][0] > 0:
        results += [score(cfg) for cfg in stage2(results[0][1])]
        results.sort(key=lambda r: -r[0])
    if results[0][0] <= 0:
        return 0.0, None, results
    return results[0][0], results[0][1], results


def check_bits(lf, torch, Hs, Hts, best, what):
    for H, Ht in zip(Hs, Hts):
        ref = torch.empty_like(H)
        lf.compute_Ht_into(H, ref)                     # built-in default
        lf.compute_Ht_into(H, Ht, config=best)
        torch.cuda.synchronize()
        if not same_bits(torch, Ht, ref):
            raise RuntimeError(f"{what} ({list(H.shape)}): the winning configuration's H' differs from the "
                               "default's")


def tune_shapes(lf, torch, shapes, esize, reps, robust):
    """Tune over `shapes` (one dtype); robust: the class rules (floor and
    minimum gain against the built-in default)."""
    dt = torch.float32 if esize == 4 else torch.float16
    Hs = [random_psf(torch, s, dt) for s in shapes]
    Hts = [torch.empty_like(H) for H in Hs]
    runs = [((lambda c, H=H, Ht=Ht: lf.compute_Ht_into(H, Ht, config=c)), 2 * H.numel() * H.element_size())
            for H, Ht in zip(Hs, Hts)]
    default = [nb / _time(lambda: run(None), torch, reps) / 1e9 for run, nb in runs]
    floor = [MAX_LOSS * d for d in default] if robust else None
    best_gbs, best, results = sweep(runs, torch, reps, 5, False, floor)
    kept_default = best is None or (robust and best_gbs < MIN_GAIN * geomean(default))
    if kept_default:
        best, best_gbs = {}, geomean(default)
    check_bits(lf, torch, Hs, Hts, best, "tuning")
    full = full_config(lf, shapes[0], dt, best)
    info = {"shapes": [list(s) for s in shapes], "esize": esize, "best_gbs": round(best_gbs, 1),
            "best_per_shape": results[0][2] if not kept_default else [round(r, 1) for r in default],
            "config": full, "default_gbs": round(geomean(default), 1),
            "default_per_shape": [round(r, 1) for r in default], "kept_default": kept_default,
            "runner_up": [(round(g, 1), c) for g, c, _ in results[1:4]]}
    del Hs, Hts
    torch.cuda.empty_cache()
    return [full[f] for f in FIELDS], info


def tune_class(lf, torch, esize, cls, reps):
    vals, info = tune_shapes(lf, torch, CLASS_SHAPES[(esize, cls)], esize, reps, True)
    info["class"] = [esize, cls]
    return ("class", 0, esize, cls), vals, info


def tune_named(lf, torch, name, reps):
    shape, esize = SHAPE_WORKLOADS[name]
    vals, info = tune_shapes(lf, torch, [shape], esize, reps, False)
    info["workload"] = name
    return ("shape", 0, esize, *shape), vals, info


def tune_batched(lf, torch, lfsynth, reps):
    Hs = [random_psf(torch, w.shape, torch.float32) for w in lfsynth.BATCHED_SETS]
    outs = [torch.empty_like(h) for h in Hs]
    nbytes = sum(2 * h.numel() * 4 for h in Hs)
    best_gbs, best, results = sweep([(lambda c: lf.compute_Ht_batched(Hs, outs, config=c), nbytes)], torch,
                                    max(3, reps // 2), 2, True)
    if best is None:
        best = {}
    refs = [torch.empty_like(h) for h in Hs]
    for h, r in zip(Hs, refs):
        lf.compute_Ht_into(h, r)
    lf.compute_Ht_batched(Hs, outs, config=best)
    torch.cuda.synchronize()
    if not all(same_bits(torch, o, r) for o, r in zip(outs, refs)):
        raise RuntimeError("batched: the winning configuration's H' differs from the plain calls'")
    lf.release_plans()
    big = max(lfsynth.BATCHED_SETS, key=lambda w: w.elements)
    full = full_config(lf, big.shape, torch.float32, best)
    key = ("shape", 1, 4, *big.shape)
    return key, [full[f] for f in FIELDS], {"workload": "batched", "best_gbs": round(best_gbs, 1), "config": full,
                                            "runner_up": [(round(g, 1), c) for g, c, _ in results[1:4]]}


def time_shapes(lf, torch, spec: str, reps: int):
    """Rate of the library's own choice on each shape of spec."""
    out = []
    for item in spec.split(";"):
        dims, _, dts = item.partition(":")
        shape = tuple(int(v) for v in dims.split(","))
        dt = torch.float16 if dts == "f16" else torch.float32
        H = random_psf(torch, shape, dt)
        Ht = torch.empty_like(H)
        t = _time(lambda: lf.compute_Ht_into(H, Ht), torch, reps)
        out.append({"shape": list(shape), "dtype": "f16" if dt == torch.float16 else "f32",
                    "row_class": row_class(shape, H.element_size()), "config": lf.default_config(shape, dt),
                    "GBs": round(2 * H.numel() * H.element_size() / t / 1e9, 1)})
        del H, Ht
        torch.cuda.empty_cache()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--classes", default=",".join(f"{'f32' if e == 4 else 'f16'}:{c}" for e, c in CLASS_SHAPES))
    ap.add_argument("--shapes", default=",".join(SHAPE_WORKLOADS))
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--reps", type=int, default=7)
    ap.add_argument("--time-shapes", default=None)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    if args.time_shapes:
        import torch
        import paper_2003_09133_amd as lf
        print(json.dumps(time_shapes(lf, torch, args.time_shapes, args.reps)), flush=True)
        return
    if args.batched_only:
        # child process: the library has read the plain entries from $LFBP_TUNE_TABLE
        import torch
        import lfsynth
        import paper_2003_09133_amd as lf
        entries = read_table(args.out)
        key, vals, info = tune_batched(lf, torch, lfsynth, args.reps)
        entries[key] = vals
        print(json.dumps(info), flush=True)
        write_table(args.out, entries, [f"batched: {info['best_gbs']} GB/s on {torch.cuda.get_device_name(0)}"])
        return
    # Tune the plain classes against the built-in defaults, not an older table.
    os.environ["LFBP_TUNE_TABLE"] = os.path.join(HERE, "_no_table_")
    import torch
    import paper_2003_09133_amd as lf

    entries = kept_entries(read_table(args.out), not args.no_batched)
    old_notes = [n for n in read_notes(args.out) if args.no_batched or not n.startswith("batched:")]
    notes = []
    dev = torch.cuda.get_device_name(0)
    for name in args.shapes.split(","):
        if not name:
            continue
        key, vals, info = tune_named(lf, torch, name, args.reps)
        entries[key] = vals
        notes.append(f"{name} {info['shapes'][0]}: {info['best_gbs']} GB/s (built-in default "
                     f"{info['default_gbs']}) on {dev}")
        print(json.dumps(info), flush=True)
    for item in args.classes.split(","):
        if not item:
            continue
        dts, _, cls = item.partition(":")
        esize = 2 if dts == "f16" else 4
        key, vals, info = tune_class(lf, torch, esize, int(cls), args.reps)
        entries[key] = vals
        notes.append(f"{dts} class {cls}: {info['best_gbs']} GB/s geometric mean over {info['shapes']} "
                     f"(built-in default {info['default_gbs']}{', kept' if info['kept_default'] else ''}) on {dev}")
        print(json.dumps(info), flush=True)
    notes = merge_notes(old_notes, notes)
    write_table(args.out, entries, notes)
    if not args.no_batched:
        env = dict(os.environ, LFBP_TUNE_TABLE=args.out)
        r = subprocess.run([sys.executable, "-m", "paper_2003_09133_amd.autotune", "--batched-only", "--out",
                            args.out, "--reps", str(args.reps)], env=env, cwd=os.path.dirname(HERE))
        if r.returncode != 0:
            raise SystemExit(r.returncode)
        # keep the plain notes beside the batched one
        entries = read_table(args.out)
        with open(args.out) as fh:
            bnotes = [l[2:].strip() for l in fh if l.startswith("# batched:")]
        write_table(args.out, entries, notes + bnotes)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
