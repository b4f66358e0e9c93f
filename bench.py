#!/usr/bin/env python3
"""Benchmark of the H' build (and its batched and projector forms) on one GPU.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline] [--no-extras]

Prints ONE JSON line.  The default workload is the camera PSF
H[345,345,15,15,51] in float32, the largest single-GPU configuration; its line
also carries, measured in the same run, the camera PSF in float16 storage, the
microscope PSF, the 16-set batched table against 16 per-set launches
(minimum and median step times of both), the projector pair, the
Richardson-Lucy update, the gradient with respect to H, the in-place build and
the column-major Table 1 sizes (each as its own line times it), and, from the
oracle leg, a bit-exact
comparison of every timed output with the CPU oracle (whole arrays for the
float32 PSFs, samples for the others).

A step is one pass of the hot path over its synthetic
input, already resident in HBM: one lfbp_compute_Ht call (plain workloads), one
lfbp_compute_Ht_batched call over a table of PSF sets (batched, batched-small),
one forward plus one backward projection (projector), one Richardson-Lucy
update (rl), one gradient with respect to H (grad-psf), or one
lfbp_compute_Ht_colmajor call per size of Table 1 on column-major arrays
(table1).  K steps are timed with HIP events
on the stream the kernels run on, bracketed by device synchronisation.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H' build GB/s & % HBM peak (bit-exact); batched vs per-PSF speedup"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, public spec
FP32_PEAK_TFLOPS = 157.3       # MI355X dense FP32 (vector and matrix)
PLAIN = {"tiny": ("TINY", "f32"), "microscope": ("MICROSCOPE", "f32"), "camera": ("CAMERA", "f32"),
         "camera-f16": ("CAMERA", "f16")}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="camera",
                    choices=sorted(PLAIN) + ["batched", "batched-small", "projector", "rl", "grad-psf", "table1"])
    ap.add_argument("--variant", default=None, choices=[None, "direct", "staged"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="camera workload: skip the figures of the other workloads")
    ap.add_argument("--inplace", action="store_true",
                    help="plain workloads: time lfbp_compute_Ht_inplace (H' written over H)")
    ap.add_argument("--copy", action="store_true",
                    help="time a plain device-to-device copy of the same bytes instead (reference ceiling)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time budget of the oracle baseline")
    return ap.parse_args()


def kernel_source_sha() -> str:
    """Digest of everything that decides which gather kernel runs and how."""
    h = hashlib.sha256()
    for f in ("csrc/lfbp_gather.hip", "csrc/lfbp_internal.h", "csrc/lfbp_api.cpp", "csrc/lfbp_tune.cpp",
              "lfbp_tune.txt"):
        with open(os.path.join(ROOT, "paper_2003_09133_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def projector_source_sha() -> str:
    """Digest of the projector kernels and their launch code."""
    h = hashlib.sha256()
    for f in ("csrc/lfbp_project.hip", "csrc/lfbp_internal.h", "csrc/lfbp_api_project.cpp"):
        with open(os.path.join(ROOT, "paper_2003_09133_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def inplace_source_sha() -> str:
    """Digest of the in-place kernel and its launch code."""
    h = hashlib.sha256()
    for f in ("csrc/lfbp_inplace.hip", "csrc/lfbp_internal.h"):
        with open(os.path.join(ROOT, "paper_2003_09133_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def inplace_traffic(workload: str):
    """HBM bytes of one in-place launch from the committed counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"inplace_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha") != inplace_source_sha():
        return None
    return t.get("hbm_bytes_per_launch")


def colmajor_source_sha() -> str:
    """Digest of the column-major kernel and its launch code."""
    h = hashlib.sha256()
    for f in ("csrc/lfbp_colmajor.hip", "csrc/lfbp_internal.h"):
        with open(os.path.join(ROOT, "paper_2003_09133_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def colmajor_traffic(shape):
    """HBM bytes of one column-major launch on `shape` from the committed
    counter summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "colmajor_table1_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha") != colmajor_source_sha():
        return None
    return t.get("shapes", {}).get("x".join(map(str, shape)), {}).get("hbm_bytes_per_launch")


def projector_traffic():
    """HBM bytes of one forward GEMM launch from the committed counter summary,
    if it was taken on the current projector source; else None."""
    path = os.path.join(ROOT, "profiles", "projector_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha") != projector_source_sha():
        return None
    kern = t.get("kernels", {})
    return kern.get("k_fwd16", kern.get("k_gemm<0>", {})).get("hbm_bytes_per_launch")


def step_traffic(workload: str):
    """HBM bytes of one step (every kernel of one update or gradient) from the
    committed counter summary of a projector-family workload, if it was taken
    on the current projector source; else None."""
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha") != projector_source_sha():
        return None
    return t.get("hbm_bytes_per_step")


def traffic_from_profile(workload: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"gather_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha") != kernel_source_sha():
        return None
    return t.get("hbm_bytes_per_launch")


def cores_used() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def time_steps(fn, steps, warmup, torch):
    """Total seconds of `steps` back-to-back calls of fn on the current stream
    (HIP events), and the wall time around them."""
    total, wall, _ = time_each(fn, steps, warmup, torch)
    return total, wall


def time_each(fn, steps, warmup, torch):
    """`steps` back-to-back calls of fn with a HIP event recorded on the
    current stream between consecutive calls: (total seconds, wall seconds,
    per-step seconds)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [ev[i].elapsed_time(ev[i + 1]) / 1000.0 for i in range(steps)]
    return ev[0].elapsed_time(ev[steps]) / 1000.0, wall, per


def time_flushed(fn, steps, warmup, torch, mode):
    """`steps` calls of fn, each after a 1 GiB buffer is written (mode
    "written": the 256 MB MALL then holds dirty lines of the buffer, which the
    call must evict) or read ("read": it holds clean lines only), with HIP
    events around each call alone.  Returns the per-call seconds."""
    buf = torch.empty(1 << 28, dtype=torch.float32, device=torch.device("cuda:0"))
    buf.zero_()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = []
    for i in range(steps):
        if mode == "written":
            buf.fill_(float(i))
        else:
            buf.sum()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        evs.append((e0, e1))
    torch.cuda.synchronize()
    del buf
    torch.cuda.empty_cache()
    return [a.elapsed_time(b) / 1000.0 for a, b in evs]


def memcpy_figures(torch, nbytes, steps, warmup):
    """hipMemcpyAsync device to device of nbytes on the current stream (the
    HIP runtime's own copy, as a ceiling for a read-once write-once pass):
    GB/s of (read + write) over `steps` back-to-back copies."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpyAsync.restype = ctypes.c_int
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    dev = torch.device("cuda:0")
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    src.fill_(7)
    stream = torch.cuda.current_stream().cuda_stream
    status = []

    def step():
        status.append(hip.hipMemcpyAsync(dst.data_ptr(), src.data_ptr(), nbytes, 3, stream))  # device to device

    total, _, per = time_each(step, steps, warmup, torch)
    ok = all(r == 0 for r in status) and bool(torch.equal(dst[:4096], src[:4096]))
    del src, dst
    torch.cuda.empty_cache()
    return {"GBs": round(2 * nbytes / (total / steps) / 1e9, 1), "step_ms": spread_ms(per), "ok": ok}


def device_figures(torch):
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
            "memory_GiB": round(p.total_memory / 2**30, 1)}


def flushed_figures(torch, lf, H, steps, warmup):
    """The plain build of H timed after a 1 GiB buffer is written and after it
    is read: GB/s at the median call and the call-time spread, per mode."""
    dH = torch.from_numpy(H).to(torch.device("cuda:0"))
    dHt = torch.empty_like(dH)
    out = {}
    for mode in ("written", "read"):
        per = time_flushed(lambda: lf.compute_Ht_into(dH, dHt), steps, warmup, torch, mode)
        med = sorted(per)[len(per) // 2]
        out[mode] = {"GBs_at_median": round(2 * H.nbytes / med / 1e9, 1), "step_ms": spread_ms(per)}
    del dH, dHt
    torch.cuda.empty_cache()
    return out


def spread_ms(per):
    """min / median / mean of per-step seconds, in ms."""
    import statistics
    return {"min": round(min(per) * 1e3, 4), "median": round(statistics.median(per) * 1e3, 4),
            "mean": round(sum(per) / len(per) * 1e3, 4)}


def cpu_oracle_rate(H, nthreads, budget_s):
    """Oracle H' on the host: GB/s of (read + write) on whole passes over H,
    repeated until about budget_s seconds have passed (after one untimed
    pass).  Returns (GB/s, timed passes, seconds per pass, the oracle's H')."""
    import numpy as np
    import oracle
    out = np.empty_like(H)
    oracle.Ht_rows(H, nthreads=nthreads, out=out)
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.Ht_rows(H, nthreads=nthreads, out=out)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = (time.perf_counter() - t0) / reps
    return 2.0 * H.nbytes / dt / 1e9, reps, dt, out


def budget_sample(run, pilot_n, total_n, budget_s):
    """Time run(n) on a pilot of pilot_n items, then on as many items as fill
    about budget_s seconds (at most total_n).  Returns (items, seconds) of the
    second run."""
    t0 = time.perf_counter()
    run(pilot_n)
    pilot = max(time.perf_counter() - t0, 1e-4)
    n = int(min(total_n, max(pilot_n, pilot_n * budget_s / pilot)))
    t0 = time.perf_counter()
    run(n)
    return n, time.perf_counter() - t0


def paper_method_rates(H, nthreads):
    """The paper's own method (oracle.paper_Ht: Eqs. 4-9 looped as in Fig. 10)
    on the host, one pass on one core and one on `nthreads`: GB/s of (read +
    write) of H's bytes."""
    import numpy as np
    import oracle
    out = np.zeros_like(H)
    rates = {}
    for n in (1, nthreads):
        t0 = time.perf_counter()
        oracle.paper_Ht(H, nthreads=n, out=out)
        rates[n] = 2.0 * H.nbytes / (time.perf_counter() - t0) / 1e9
    return rates


def _bits(a):
    import numpy as np
    return a.view(np.uint32 if a.dtype.itemsize == 4 else np.uint16)


def oracle_parity(checks, nthreads, full_ref=None):
    """Bit-exact comparison of the timed GPU outputs with the oracle.  Each
    check is (name, H, idx, got): idx None means `got` is the whole H' (compared
    with the oracle's whole H', or with `full_ref[name]` when the timing passes
    already produced it), else `got` holds H' at the flat indices idx."""
    import numpy as np
    import oracle
    res = {}
    for name, H, idx, got in checks:
        if idx is None:
            ref = (full_ref or {}).get(name)
            if ref is None:
                ref = oracle.Ht_rows(H, nthreads=nthreads)
            bad = int(np.count_nonzero(_bits(ref).ravel() != _bits(got).ravel()))
            res[name] = {"compared": f"all {got.size} elements", "mismatches": bad}
        else:
            ref = oracle.Ht_at(H, idx, nthreads=nthreads)
            bad = int(np.count_nonzero(_bits(ref) != _bits(got)))
            res[name] = {"compared": f"{idx.size} sampled elements", "mismatches": bad}
    return res


def gather_run(torch, lf, H, steps, warmup, config=None):
    """Upload H, then time `steps` lfbp_compute_Ht calls into one output.
    Returns (total s, wall s, per-step s, output tensor on the GPU)."""
    dH = torch.from_numpy(H).to(torch.device("cuda:0"))
    dHt = torch.empty_like(dH)
    total, wall, per = time_each(lambda: lf.compute_Ht_into(dH, dHt, config=config), steps, warmup, torch)
    del dH
    return total, wall, per, dHt


def gpu_sample(torch, t, idx):
    """Elements of GPU tensor t at flat indices idx, copied to the host."""
    return t.view(-1)[torch.from_numpy(idx).to(t.device)].cpu().numpy()


def batched_vs_sequential(args, torch, lf, lfsynth, sets, rng):
    """The batched call against one plain call per set, timed step by step on
    the same tensors.  Returns (figures, checks for the oracle leg)."""
    import numpy as np
    from paper_2003_09133_amd import _abi

    dev = torch.device("cuda:0")
    Hs_host, Hs, Hts = [], [], []
    for w in sets:
        H, _ = lfsynth.make_H(w)
        Hs_host.append(H)
        Hs.append(torch.from_numpy(H).to(dev))
        Hts.append(torch.empty_like(Hs[-1]))
    nbytes = sum(2 * h.numel() * h.element_size() for h in Hs)
    batched = lf.BatchedHt(Hs, Hts)
    batched_graph = lf.BatchedHt(Hs, Hts, use_graph=True)
    batched_persist = lf.BatchedHt(Hs, Hts, config={"persistent": 1})
    L = _abi.lib()
    plain_args = [(h.data_ptr(), o.data_ptr(), _abi.Shape.of(h.shape)) for h, o in zip(Hs, Hts)]
    stream = torch.cuda.current_stream().cuda_stream

    def sequential():
        for hp, op, shp in plain_args:
            L.lfbp_compute_Ht(hp, op, shp, _abi.F32, stream)

    # two alternating rounds of each form, so that slow drifts of the clock or
    # the memory state fall on both
    per_seq, per_bat = [], []
    for _ in range(2):
        per_seq += time_each(sequential, args.steps, args.warmup, torch)[2]
        per_bat += time_each(batched, args.steps, args.warmup, torch)[2]
    # the 16 plain calls captured once into one graph by the caller and
    # replayed (no launch gaps between them)
    seq_graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(seq_graph):
        cap = torch.cuda.current_stream().cuda_stream
        for hp, op, shp in plain_args:
            if L.lfbp_compute_Ht(hp, op, shp, _abi.F32, cap) != 0:
                raise RuntimeError("lfbp_compute_Ht failed during graph capture")
    per_seqg = time_each(seq_graph.replay, args.steps, args.warmup, torch)[2]
    del seq_graph
    # the same table replayed from the plan's captured graph, and the
    # persistent (pipelined) kernel, beside the default direct launch
    per_graph = time_each(batched_graph, args.steps, args.warmup, torch)[2]
    per_pers = time_each(batched_persist, args.steps, args.warmup, torch)[2]
    lf.release_plans()
    checks = []
    for i, (H, o) in enumerate(zip(Hs_host, Hts)):          # outputs of the last (batched, persistent) call
        idx = rng.integers(0, H.size, 200_000)
        checks.append((f"batched set {i} {list(H.shape)}", H, idx, gpu_sample(torch, o, idx)))
    del Hs, Hts, batched, batched_graph, batched_persist
    s_seq, s_bat = spread_ms(per_seq), spread_ms(per_bat)
    figures = {
        "sets": len(sets), "bytes_per_step": nbytes, "steps_per_form": len(per_bat),
        "batched_ms": s_bat, "sequential_ms": s_seq,
        "sequential_in_one_graph_ms": spread_ms(per_seqg),
        "batched_graph_replay_ms": spread_ms(per_graph), "batched_persistent_ms": spread_ms(per_pers),
        "batched_GBs_median": round(nbytes / (s_bat["median"] * 1e-3) / 1e9, 1),
        "speedup_median": round(s_seq["median"] / s_bat["median"], 4),
        "speedup_vs_sequential_in_one_graph_median": round(spread_ms(per_seqg)["median"] / s_bat["median"], 4),
        "speedup_min": round(s_seq["min"] / s_bat["min"], 4),
        "speedup_mean": round(s_seq["mean"] / s_bat["mean"], 4),
    }
    return figures, checks


def other_lines(args, torch):
    """The projector pair, the Richardson-Lucy update, the gradient with
    respect to H, the in-place build of the camera PSF and the column-major
    Table 1 sizes, each run as its own workload line runs it (same steps and
    warm-up, no CPU leg), summarised by value, step time and roofline."""
    runs = (("projector-pair", "projector", False, bench_projector), ("rl-update", "rl", False, bench_rl),
            ("grad-psf", "grad-psf", False, bench_grad_psf), ("inplace-camera", "camera", True, bench_plain),
            ("colmajor-table1", "table1", False, bench_table1))
    res = {}
    for name, workload, inplace, fn in runs:
        sub = argparse.Namespace(**vars(args))
        sub.workload, sub.inplace, sub.no_cpu_baseline, sub.no_extras = workload, inplace, True, True
        d = fn(sub, torch)
        res[name] = {"workload": d["config"]["workload"], "value": d["value"], "unit": d["unit"],
                     "ms_per_step": d["ms_per_step"], "roofline": d["roofline"]}
        torch.cuda.empty_cache()
    return res


def bench_plain(args, torch):
    import numpy as np
    import lfsynth
    import paper_2003_09133_amd as lf

    wname, dt = PLAIN[args.workload]
    w = getattr(lfsynth, wname)
    npdt = np.float32 if dt == "f32" else np.float16
    H, zf = lfsynth.make_H(w, npdt)
    dev = torch.device("cuda:0")
    cfg = None
    if args.variant:
        cfg = {"variant": lf.GATHER_DIRECT if args.variant == "direct" else lf.GATHER_STAGED}
    resolved = lf.default_config(w.shape, torch.float32 if dt == "f32" else torch.float16)
    if cfg:
        resolved.update(cfg)
    got = None
    if args.copy or args.inplace:
        dH = torch.from_numpy(H).to(dev)
        if args.copy:
            dHt = torch.empty_like(dH)
            step = lambda: dHt.copy_(dH)
        else:
            step = lambda: lf.compute_Ht_inplace(dH)     # each step undoes the previous one (involution)
        elapsed, wall, per = time_each(step, args.steps, args.warmup, torch)
    else:
        elapsed, wall, per, dHt = gather_run(torch, lf, H, args.steps, args.warmup, cfg)
        got = dHt.cpu().numpy()
        del dHt
    torch.cuda.empty_cache()
    bytes_step = 2 * H.nbytes
    sec_step = elapsed / args.steps
    gbs = bytes_step / sec_step / 1e9
    out = {
        "metric": METRIC, "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec_step * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dt, "data": "synthetic",
        "config": {"workload": f"{w.name} H{list(w.shape)} {dt}", "shape": list(w.shape),
                   "bytes_per_step": bytes_step, "zero_fraction": round(zf, 4), "step_ms": spread_ms(per),
                   "device": device_figures(torch),
                   "kernel": ("torch copy_ (reference)" if args.copy else
                              "k_inplace (H' over H)" if args.inplace else resolved), "wall_s": round(wall, 3)},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": (None if args.copy else inplace_traffic(args.workload) if args.inplace
                                 else traffic_from_profile(args.workload))},
    }
    checks = [] if got is None else [(out["config"]["workload"], H, None, got)]
    if args.workload == "microscope" and not (args.copy or args.inplace):
        # H and H' (0.5 GB each) are twice the 256 MB MALL: also timed with the cache state between calls
        # set by a 1 GiB buffer
        out["config"]["after_1GiB_buffer"] = flushed_figures(torch, lf, H, args.steps, args.warmup)
    if args.workload == "camera" and not (args.copy or args.inplace or args.no_extras):
        rng = np.random.default_rng(2003)
        also = {}
        # the same PSF in float16 storage
        H16 = H.astype(np.float16)
        t16, _, per16, d16 = gather_run(torch, lf, H16, args.steps, args.warmup)
        idx = rng.integers(0, H16.size, 2_000_000)
        checks.append((f"{w.name} H{list(w.shape)} f16", H16, idx, gpu_sample(torch, d16, idx)))
        del d16
        torch.cuda.empty_cache()
        g16 = 2 * H16.nbytes / (t16 / args.steps) / 1e9
        also["camera-f16"] = {"GBs": round(g16, 1), "frac": round(g16 / HBM_PEAK_GBS, 4), "step_ms": spread_ms(per16),
                              "traffic": traffic_from_profile("camera-f16")}
        # the microscope PSF (1 GB per step: partly held by the 256 MB MALL between steps)
        mw = lfsynth.MICROSCOPE
        Hm, _ = lfsynth.make_H(mw)
        tm, _, perm, dm = gather_run(torch, lf, Hm, args.steps, args.warmup)
        checks.append((f"{mw.name} H{list(mw.shape)} f32", Hm, None, dm.cpu().numpy()))
        del dm
        torch.cuda.empty_cache()
        gm = 2 * Hm.nbytes / (tm / args.steps) / 1e9
        also["microscope"] = {"GBs": round(gm, 1), "frac": round(gm / HBM_PEAK_GBS, 4), "step_ms": spread_ms(perm),
                              "traffic": traffic_from_profile("microscope"),
                              "after_1GiB_buffer": flushed_figures(torch, lf, Hm, args.steps, args.warmup)}
        # the HIP runtime's device-to-device copy of the same bytes
        mc = memcpy_figures(torch, H.nbytes, args.steps, args.warmup)
        mc["gather_over_memcpy"] = round(gbs / mc["GBs"], 4)
        also["hipMemcpyAsync-d2d"] = mc
        # 16 PSF sets: one batched launch against 16 per-set launches
        also["batched-16"], bchecks = batched_vs_sequential(args, torch, lf, lfsynth, lfsynth.BATCHED_SETS, rng)
        checks += bchecks
        torch.cuda.empty_cache()
        # the rest of the path, each timed as its own line does (without its CPU leg)
        also.update(other_lines(args, torch))
        out["config"]["also"] = also
    if not args.no_cpu_baseline and not args.copy and not args.inplace:
        nth = cores_used()
        rate, passes, per_pass, ref = cpu_oracle_rate(H, nth, args.cpu_seconds)
        out["cpu_baseline"] = {"value": round(rate, 3), "unit": "GB/s", "cores": nth, "kind": "oracle",
                               "sample": f"{passes} full passes of the oracle over the same H "
                                         f"({per_pass:.3g} s each, {passes * per_pass:.1f} s in all)"}
        if args.workload == "camera":
            pm = paper_method_rates(H, nth)
            out["cpu_baseline"]["paper_method"] = {
                "GBs_1_core": round(pm[1], 3), f"GBs_{nth}_cores": round(pm[nth], 3),
                "sample": "one pass of the paper's method (Eqs. 4-9 looped as in Fig. 10, C) over the same H "
                          "on each core count"}
        out["config"]["bit_exact_vs_oracle"] = oracle_parity(checks, nth, {out["config"]["workload"]: ref})
    return out


def bench_batched(args, torch):
    import numpy as np
    import lfsynth
    import paper_2003_09133_amd as lf

    small = args.workload == "batched-small"
    sets = lfsynth.SMALL_SETS if small else lfsynth.BATCHED_SETS
    dev = torch.device("cuda:0")
    Hs, Hts = [], []
    for w in sets:
        H, _ = lfsynth.make_H(w)
        Hs.append(torch.from_numpy(H).to(dev))
        Hts.append(torch.empty_like(Hs[-1]))
        del H
    bytes_step = sum(2 * h.numel() * 4 for h in Hs)

    # Every form with its arguments prepared once, so that each step is C
    # calls only: one batched call (a direct launch, the default, or a replay
    # of the plan's captured graph), or one plain call per set.
    from paper_2003_09133_amd import _abi
    batched = lf.BatchedHt(Hs, Hts)
    batched_graph = lf.BatchedHt(Hs, Hts, use_graph=True)
    batched_persist = lf.BatchedHt(Hs, Hts, config={"persistent": 1})
    L = _abi.lib()
    plain_args = [(h.data_ptr(), o.data_ptr(), _abi.Shape.of(h.shape)) for h, o in zip(Hs, Hts)]
    stream = torch.cuda.current_stream().cuda_stream

    def sequential():
        for hp, op, shp in plain_args:
            L.lfbp_compute_Ht(hp, op, shp, _abi.F32, stream)

    t_seq, _ = time_steps(sequential, args.steps, args.warmup, torch)
    # the same per-set calls captured once into a graph by the caller and
    # replayed (no launch gaps between them)
    seq_graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(seq_graph):
        cap = torch.cuda.current_stream().cuda_stream
        for hp, op, shp in plain_args:
            if L.lfbp_compute_Ht(hp, op, shp, _abi.F32, cap) != 0:
                raise RuntimeError("lfbp_compute_Ht failed during graph capture")
    t_seqg, _ = time_steps(seq_graph.replay, args.steps, args.warmup, torch)
    t_graph, _ = time_steps(batched_graph, args.steps, args.warmup, torch)
    t_pers, _ = time_steps(batched_persist, args.steps, args.warmup, torch)
    t_bat, wall = time_steps(batched, args.steps, args.warmup, torch)
    sec = t_bat / args.steps
    gbs = bytes_step / sec / 1e9
    out = {
        "metric": METRIC, "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": ("batched 64 small PSF sets f32 (Nnum 3-7, 3-7 lenslets, nz 4-12)" if small else
                                "batched 16 PSF sets f32 (Nnum 7-19, 9-25 lenslets, nz 9-41)"),
                   "bytes_per_step": bytes_step, "sets": [list(w.shape) for w in sets],
                   "sequential_ms_per_step": round(t_seq / args.steps * 1e3, 4),
                   "sequential_in_one_graph_ms_per_step": round(t_seqg / args.steps * 1e3, 4),
                   "batched_graph_replay_ms_per_step": round(t_graph / args.steps * 1e3, 4),
                   "batched_persistent_ms_per_step": round(t_pers / args.steps * 1e3, 4),
                   "batched_vs_sequential_speedup": round(t_seq / t_bat, 4),
                   "batched_vs_sequential_in_one_graph_speedup": round(t_seqg / t_bat, 4),
                   "wall_s": round(wall, 3)},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": None if small else traffic_from_profile("batched")},
    }
    return out


def bench_projector(args, torch):
    """One step = forward projection f = H g plus the backprojection of f
    through the GPU-built H' (the two products of one gradient evaluation), on
    a prepared operator (H and H' packed once, as for any run of projections
    with one PSF).  The time to prepare the operator and the pair time of the
    unprepared calls, which pack H and H' on every call, are reported beside."""
    import numpy as np
    import lfsynth
    import paper_2003_09133_amd as lf

    pw = lfsynth.PROJECTOR
    H, _ = lfsynth.make_H(pw.psf)
    R, C = pw.image
    dev = torch.device("cuda:0")
    dH = torch.from_numpy(H).to(dev)
    dHt = lf.compute_Ht(dH)
    g = torch.from_numpy(lfsynth.uniform_f32((pw.psf.shape[4], R, C), pw.g_seed)).to(dev)
    f = torch.empty((R, C), device=dev)
    gb = torch.empty_like(g)
    # scratch for the operand records, allocated once as an iterative solver would
    wf = torch.empty(lf.forward_workspace_size(H.shape, R, C), dtype=torch.uint8, device=dev)
    wb = torch.empty(lf.backward_workspace_size(H.shape, R, C), dtype=torch.uint8, device=dev)
    fwd_plain = lambda: lf.forward(dH, g, out=f, workspace=wf)
    bwd_plain = lambda: lf.backward(dHt, f, out=gb, workspace=wb)

    def step_plain():
        fwd_plain()
        bwd_plain()

    t_plain, _ = time_steps(step_plain, args.steps, args.warmup, torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = lf.LFOperator(dH, R, C, Ht=dHt)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0
    fwd = lambda: op.forward(g, out=f)
    bwd = lambda: op.backward(f, out=gb)

    def step():
        fwd()
        bwd()

    t_fwd, _ = time_steps(fwd, args.steps, args.warmup, torch)
    t_bwd, _ = time_steps(bwd, args.steps, args.warmup, torch)
    elapsed, wall = time_steps(step, args.steps, args.warmup, torch)
    sec = elapsed / args.steps
    ns, nt, nx, ny, nz = pw.psf.shape
    flop_proj = 2.0 * nz * R * C * ns * nt         # multiply-adds of one projection, no edge clipping
    tflops_fwd = flop_proj / (t_fwd / args.steps) / 1e12
    out = {
        "metric": "projections/s (forward + backprojection pair)", "value": round(1.0 / sec, 2),
        "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"projector {R}x{C} px, {pw.lenslets}x{pw.lenslets} lenslets, "
                               f"H{list(pw.psf.shape)} f32",
                   "forward_ms": round(t_fwd / args.steps * 1e3, 4),
                   "backward_ms": round(t_bwd / args.steps * 1e3, 4),
                   "prepared_operator": True, "prepare_ms": round(t_prep * 1e3, 3),
                   "unprepared_ms_per_step": round(t_plain / args.steps * 1e3, 4),
                   "flop_per_projection": flop_proj, "wall_s": round(wall, 3)},
        "roofline": {"bound": "mfma", "achieved": round(tflops_fwd, 2), "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(tflops_fwd / FP32_PEAK_TFLOPS, 4),
                     "traffic": projector_traffic()},
    }
    if not args.no_cpu_baseline:
        import oracle
        nth = cores_used()
        rng = np.random.default_rng(0)
        pix = rng.integers(0, [R, C], size=(R * C, 2))
        gh = g.cpu().numpy()
        n, dt = budget_sample(lambda k: oracle.forward_at(H, gh, pix[:k], nthreads=nth), 400, R * C,
                              args.cpu_seconds)
        per_proj = dt * (R * C) / n
        out["cpu_baseline"] = {"value": round(1.0 / (2 * per_proj), 6), "unit": "pairs/s", "cores": nth,
                               "kind": "oracle", "sample": f"float64 oracle forward at {n} random pixels "
                                                           f"({dt:.2f} s), scaled to a full forward+backward pair"}
    return out


def bench_rl(args, torch):
    """One step = one Richardson-Lucy update (Eq. 2) of a 21 x 600 x 600 volume
    from a 600 x 600 shot-noise image (Poisson counts, 50 photons per pixel on
    average): forward projection ending in the quotient,
    backprojection through H' ending in the update, on an operator prepared
    once as richardson_lucy does (lfbp_rl_step_op).  The preparation time and
    the step time of lfbp_rl_step, which packs H and H' on every call, are
    reported beside."""
    import numpy as np
    import lfsynth
    import paper_2003_09133_amd as lf

    pw = lfsynth.PROJECTOR
    H, _ = lfsynth.make_H(pw.psf)
    R, C = pw.image
    dev = torch.device("cuda:0")
    dH = torch.from_numpy(H).to(dev)
    dHt = lf.compute_Ht(dH)
    # shot-noise data f = Poisson(H g_true), 50 photons per pixel on average;
    # the noise-free image comes from the library's own forward projection
    g_true = torch.from_numpy(lfsynth.uniform_f32((pw.psf.shape[4], R, C), pw.g_seed + 1) ** 4).to(dev)
    mean = lf.forward(dH, g_true).double()
    lam = (mean * (50.0 / mean.mean())).cpu().numpy()
    f = torch.from_numpy(lfsynth.poisson_counts(lam, pw.g_seed + 2)).to(dev)
    del g_true, mean
    g = torch.ones((pw.psf.shape[4], R, C), device=dev)
    ws = torch.empty(lf.rl_workspace_size(H.shape, R, C), dtype=torch.uint8, device=dev)
    norm = lf.rl_norm(dHt, R, C, workspace=ws)
    g_plain = g.clone()
    t_plain, _ = time_steps(lambda: lf.rl_step(dH, dHt, f, g_plain, norm, out=g_plain, workspace=ws), args.steps,
                            args.warmup, torch)
    del g_plain, ws
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = lf.LFOperator(dH, R, C, Ht=dHt)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0

    def step():
        op.rl_step(f, g, norm, out=g)

    elapsed, wall = time_steps(step, args.steps, args.warmup, torch)
    sec = elapsed / args.steps
    ns, nt, nx, ny, nz = pw.psf.shape
    flop = 2 * 2.0 * nz * R * C * ns * nt          # one forward and one backprojection
    tflops = flop / sec / 1e12
    out = {
        "metric": "Richardson-Lucy iterations/s", "value": round(1.0 / sec, 2), "unit": "iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Richardson-Lucy update, {R}x{C} px, {pw.lenslets}x{pw.lenslets} lenslets, "
                               f"H{list(pw.psf.shape)} f32", "flop_per_step": flop, "wall_s": round(wall, 3),
                   "prepared_operator": True, "prepare_ms": round(t_prep * 1e3, 3),
                   "unprepared_ms_per_step": round(t_plain / args.steps * 1e3, 4),
                   "finite": bool(torch.isfinite(g).all().item())},
        "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tflops / FP32_PEAK_TFLOPS, 4), "traffic": step_traffic("rl")},
    }
    if not args.no_cpu_baseline:
        import oracle
        nth = cores_used()
        rng = np.random.default_rng(0)
        pix = rng.integers(0, [R, C], size=(R * C, 2))
        gh = g.cpu().numpy()
        n, dt = budget_sample(lambda k: oracle.forward_at(H, gh, pix[:k], nthreads=nth), 400, R * C,
                              args.cpu_seconds)
        per_step = 2 * dt * (R * C) / n
        out["cpu_baseline"] = {"value": round(1.0 / per_step, 6), "unit": "iterations/s", "cores": nth,
                               "kind": "oracle", "sample": f"float64 oracle forward at {n} random pixels "
                                                           f"({dt:.2f} s), scaled to a forward and a backward "
                                                           f"projection of the whole volume"}
    return out


def bench_grad_psf(args, torch):
    """One step = the gradient of <w, H g> with respect to H (lfbp_grad_psf)
    on the projector grid: 600 x 600 px, 21 depths, H[165,165,15,15,21]."""
    import numpy as np
    import lfsynth
    import paper_2003_09133_amd as lf

    pw = lfsynth.PROJECTOR
    shape = pw.psf.shape
    R, C = pw.image
    dev = torch.device("cuda:0")
    w = torch.from_numpy(lfsynth.uniform_f32((R, C), pw.g_seed + 2) - np.float32(0.5)).to(dev)
    g = torch.from_numpy(lfsynth.uniform_f32((shape[4], R, C), pw.g_seed)).to(dev)
    dH = torch.empty(shape, device=dev)
    ws = torch.empty(lf.grad_psf_workspace_size(shape, R, C), dtype=torch.uint8, device=dev)
    step = lambda: lf.grad_psf(w, g, shape, out=dH, workspace=ws)
    elapsed, wall = time_steps(step, args.steps, args.warmup, torch)
    sec = elapsed / args.steps
    ns, nt, nx, ny, nz = shape
    flop = 2.0 * nz * R * C * ns * nt
    tflops = flop / sec / 1e12
    out = {
        "metric": "PSF gradients/s", "value": round(1.0 / sec, 2), "unit": "gradients/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"d<w, H g>/dH, {R}x{C} px, {pw.lenslets}x{pw.lenslets} lenslets, H{list(shape)} f32",
                   "flop_per_step": flop, "wall_s": round(wall, 3)},
        "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tflops / FP32_PEAK_TFLOPS, 4), "traffic": step_traffic("grad-psf")},
    }
    if not args.no_cpu_baseline:
        import oracle
        nth = cores_used()
        total = int(np.prod(shape))
        idx = np.random.default_rng(0).integers(0, total, min(total, 50_000_000))
        wh, gh = w.cpu().numpy(), g.cpu().numpy()
        n, dt = budget_sample(lambda k: oracle.grad_psf_at(shape, wh, gh, idx[:k], nthreads=nth), 20000, idx.size,
                              args.cpu_seconds)
        per = dt * total / n
        out["cpu_baseline"] = {"value": round(1.0 / per, 6), "unit": "gradients/s", "cores": nth, "kind": "oracle",
                               "sample": f"float64 oracle at {n} random entries of dH ({dt:.2f} s), "
                                         f"scaled to the whole array"}
    return out


def table1_paper_seconds():
    """Seconds of the paper's CPU implementation for the Table 1 sizes (the
    committed fixture that transcribes Table 1)."""
    rows = {}
    with open(os.path.join(ROOT, "tests", "golden", "table1_shapes.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                p, nx, ny, sec = line.split()
                rows[(int(p), int(nx), int(ny))] = float(sec)
    return rows


def bench_table1(args, torch):
    """One step = H' of every Table 1 size (11 depths, float32), stored
    column-major as in the paper's implementation, one launch each.  The
    row-major kernel on the same arrays is timed beside it."""
    import numpy as np
    import lfsynth
    import paper_2003_09133_amd as lf

    from paper_2003_09133_amd import _abi
    L = _abi.lib()
    dev = torch.device("cuda:0")
    paper = table1_paper_seconds()
    rows, t_col, t_row, total_bytes = [], 0.0, 0.0, 0
    largest = None
    for i, key in enumerate(lfsynth.TABLE1_SHAPES):
        w = lfsynth.table1_workload(i)
        H, _ = lfsynth.make_H(w)
        dH = torch.from_numpy(H).to(dev)
        del H
        dc = dH.permute(4, 3, 2, 1, 0).contiguous().permute(4, 3, 2, 1, 0)   # column-major storage
        out_c = torch.empty_like(dc)
        out_r = torch.empty_like(dH)
        nbytes = 2 * dH.numel() * dH.element_size()
        lf.compute_Ht_colmajor(dc, out=out_c)         # argument checks once; the steps are C calls only
        lf.compute_Ht_into(dH, out_r)
        shp, stream = _abi.Shape.of(dH.shape), torch.cuda.current_stream().cuda_stream
        pc, po, pr, pq = dc.data_ptr(), out_c.data_ptr(), dH.data_ptr(), out_r.data_ptr()
        tc, _ = time_steps(lambda: L.lfbp_compute_Ht_colmajor(pc, po, shp, _abi.F32, stream), args.steps,
                           args.warmup, torch)
        tr, _ = time_steps(lambda: L.lfbp_compute_Ht(pr, pq, shp, _abi.F32, stream), args.steps, args.warmup,
                           torch)
        del dH, dc, out_c, out_r
        tc, tr = tc / args.steps, tr / args.steps
        t_col += tc
        t_row += tr
        total_bytes += nbytes
        rows.append({"shape": list(w.shape), "colmajor_ms": round(tc * 1e3, 4),
                     "colmajor_GBs": round(nbytes / tc / 1e9, 1), "rowmajor_ms": round(tr * 1e3, 4),
                     "rowmajor_GBs": round(nbytes / tr / 1e9, 1), "paper_cpu_s": paper.get(tuple(key))})
        print(f"# {w.name}: column-major {tc * 1e3:.3f} ms, row-major {tr * 1e3:.3f} ms", file=sys.stderr,
              flush=True)
        if largest is None or nbytes > largest[0]:
            largest = (nbytes, tc, list(w.shape))
    gbs = total_bytes / t_col / 1e9
    big_gbs = largest[0] / largest[1] / 1e9
    out = {
        "metric": METRIC, "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_col * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "Table 1 sizes, 11 depths, f32, column-major storage, one launch per size",
                   "bytes_per_step": total_bytes, "rowmajor_ms_per_step": round(t_row * 1e3, 4),
                   "sizes": rows},
        "roofline": {"bound": "hbm", "achieved": round(big_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(big_gbs / HBM_PEAK_GBS, 4), "traffic": colmajor_traffic(largest[2]),
                     "kernel": f"k_colmajor on {largest[2]}"},
    }
    if not args.no_cpu_baseline:
        nth = cores_used()
        w = lfsynth.table1_workload(3)
        H, _ = lfsynth.make_H(w)
        rate, passes, per, _ = cpu_oracle_rate(H, nth, args.cpu_seconds)
        out["cpu_baseline"] = {"value": round(rate, 3), "unit": "GB/s", "cores": nth, "kind": "oracle",
                               "sample": f"{passes} full passes of the (row-major) oracle over the Table 1 "
                                         f"size {list(w.shape)} ({per:.3g} s each, {passes * per:.1f} s in all)"}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    if args.workload in ("batched", "batched-small"):
        out = bench_batched(args, torch)
    elif args.workload == "projector":
        out = bench_projector(args, torch)
    elif args.workload == "rl":
        out = bench_rl(args, torch)
    elif args.workload == "grad-psf":
        out = bench_grad_psf(args, torch)
    elif args.workload == "table1":
        out = bench_table1(args, torch)
    else:
        out = bench_plain(args, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
