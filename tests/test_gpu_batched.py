"""Batched H' (one launch for many PSF arrays) against the CPU oracle."""
import numpy as np
import pytest
import torch

import lfsynth
import oracle
import paper_2003_09133_amd as lf
from gpu_util import DEV, assert_same_bits, gpu_equal_bits, sample_indices, to_dev

pytestmark = pytest.mark.gpu

BATCH_CONFIGS = [
    None,
    {"variant": lf.GATHER_WIDE, "persistent": 1, "grid": 3, "vec_per_thread": 2},
    {"variant": lf.GATHER_WIDE, "persistent": 2, "vec_per_thread": 8, "block_threads": 512},
    {"variant": lf.GATHER_STAGED, "persistent": 1, "tile_bytes": 8192},
    {"variant": lf.GATHER_STAGED, "persistent": 2},
    {"variant": lf.GATHER_DIRECT, "persistent": 1, "grid": 11, "rows_in_flight": 1},
    {"variant": lf.GATHER_WIDE, "persistent": 2, "schedule": 2, "waves_per_eu": 4},
    {"variant": lf.GATHER_WIDE, "persistent": 1, "schedule": 2, "grid": 13, "vec_per_thread": 2},
    {"variant": lf.GATHER_STAGED, "persistent": 2, "schedule": 2, "waves_per_eu": 2},
    {"variant": lf.GATHER_DIRECT, "persistent": 1, "schedule": 2, "grid": 5},
]


def mixed_shapes(seed, n):
    rng = np.random.default_rng(seed)
    odd = lambda lo, hi: int(rng.integers(lo, hi + 1)) | 1
    return [(odd(1, 61), odd(1, 61), odd(1, 13), odd(1, 13), int(rng.integers(1, 30))) for _ in range(n)]


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("use_graph", [True, False])
def test_mixed_batch_all_configs(dtype, use_graph):
    shapes = mixed_shapes(3, 9) + [(1, 1, 1, 1, 1), (63, 63, 7, 7, 9), (3, 3, 1, 3, 700)]
    Hs = [lfsynth.bits(s, i + 100, dtype) for i, s in enumerate(shapes)]
    refs = [oracle.Ht_rows(H) for H in Hs]
    dHs = [to_dev(H) for H in Hs]
    for cfg in BATCH_CONFIGS:
        outs = lf.compute_Ht_batched(dHs, config=cfg, use_graph=use_graph)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, refs)):
            assert_same_bits(o.cpu().numpy(), r, f"set {i} {shapes[i]} {cfg} graph={use_graph}")


def test_single_problem_batch_equals_plain():
    H = to_dev(lfsynth.bits((45, 39, 9, 7, 13), 5, np.float32))
    (o,) = lf.compute_Ht_batched([H])
    assert gpu_equal_bits(o, lf.compute_Ht(H))


def test_graph_replays_follow_new_data():
    """The plan (descriptor table + graph) is reused for the same table; every
    replay reads the current contents, with unrelated eager work and
    synchronisations between replays."""
    shapes = [(21, 21, 7, 7, 5), (33, 27, 11, 9, 3), (15, 15, 3, 3, 11)]
    dHs = [torch.empty(s, dtype=torch.float32, device=DEV) for s in shapes]
    outs = [torch.empty_like(h) for h in dHs]
    scratch = torch.zeros(1 << 20, device=DEV)
    for rep in range(4):
        hs = [lfsynth.bits(s, 1000 * rep + i, np.float32) for i, s in enumerate(shapes)]
        for d, h in zip(dHs, hs):
            d.copy_(torch.from_numpy(h))
        lf.compute_Ht_batched(dHs, outs, use_graph=True)
        scratch.add_(1.0)                                  # eager work between replays
        torch.cuda.synchronize()
        for o, h in zip(outs, hs):
            assert_same_bits(o.cpu().numpy(), oracle.Ht_rows(h), f"replay {rep}")
        lf.compute_Ht(dHs[0])                              # plain calls interleaved
    lf.release_plans()
    lf.compute_Ht_batched(dHs, outs, use_graph=True)
    torch.cuda.synchronize()
    assert_same_bits(outs[1].cpu().numpy(), oracle.Ht_rows(hs[1]), "after release")


def test_plain_and_batched_calls_replay_in_a_caller_graph():
    """Plain calls and a batched call without its own graph, captured by the
    caller into one torch CUDA graph: the calls allocate nothing and record
    no memset, so every replay, with eager overwrites of the inputs and
    outputs and synchronisations between replays, gives the oracle's H'."""
    from paper_2003_09133_amd import _abi
    shapes = [(21, 21, 7, 7, 5), (33, 27, 11, 9, 3), (15, 15, 3, 3, 11), (45, 39, 9, 7, 13)]
    dHs = [torch.empty(s, dtype=torch.float32, device=DEV) for s in shapes]
    plain_out = [torch.empty_like(h) for h in dHs]
    batch_out = [torch.empty_like(h) for h in dHs]
    L = _abi.lib()
    probs = (_abi.Problem * len(shapes))(*[_abi.Problem(h.data_ptr(), o.data_ptr(), _abi.Shape.of(h.shape))
                                           for h, o in zip(dHs, batch_out)])

    def calls(stream):
        for h, o in zip(dHs, plain_out):
            assert L.lfbp_compute_Ht(h.data_ptr(), o.data_ptr(), _abi.Shape.of(h.shape), _abi.F32, stream) == 0
        assert L.lfbp_compute_Ht_batched_config(probs, len(shapes), _abi.F32, None, 0, stream) == 0

    calls(torch.cuda.current_stream().cuda_stream)       # builds the batched plan before the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        calls(torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        hs = [lfsynth.bits(s, 500 * rep + i, np.float32) for i, s in enumerate(shapes)]
        for d, h in zip(dHs, hs):
            d.copy_(torch.from_numpy(h))
        for o in plain_out + batch_out:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for i, h in enumerate(hs):
            ref = oracle.Ht_rows(h)
            assert_same_bits(plain_out[i].cpu().numpy(), ref, f"replay {rep} plain set {i}")
            assert_same_bits(batch_out[i].cpu().numpy(), ref, f"replay {rep} batched set {i}")


def test_concurrent_batched_calls_from_threads():
    """Four host threads submit their own tables at the same time, each on a
    stream of its own, alternating direct launches and graph replays; the
    plan cache is shared under a lock, and every result is the oracle's (one
    table of 20 problems takes the device descriptor table)."""
    import threading
    counts = (5, 12, 20, 3)
    Hs = [[lfsynth.bits(s, 100 * k + i, np.float32) for i, s in enumerate(mixed_shapes(40 + k, n))]
          for k, n in enumerate(counts)]
    dHs = [[to_dev(h) for h in hs] for hs in Hs]
    outs = [[torch.empty_like(h) for h in hs] for hs in dHs]
    torch.cuda.synchronize()
    errors = []

    def work(k):
        try:
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                for it in range(6):
                    lf.compute_Ht_batched(dHs[k], outs[k], use_graph=bool(it % 2))
            stream.synchronize()
        except Exception as e:          # reported below, on the main thread
            errors.append((k, e))

    threads = [threading.Thread(target=work, args=(k,)) for k in range(len(counts))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    torch.cuda.synchronize()
    for k, (hs, os_) in enumerate(zip(Hs, outs)):
        for i, (h, o) in enumerate(zip(hs, os_)):
            assert_same_bits(o.cpu().numpy(), oracle.Ht_rows(h), f"thread {k} set {i}")


def test_batch_rejects_mixed_dtypes_and_overlap():
    a = torch.zeros((5, 5, 3, 3, 2), device=DEV)
    b = torch.zeros((5, 5, 3, 3, 2), device=DEV, dtype=torch.float16)
    with pytest.raises(TypeError):
        lf.compute_Ht_batched([a, b])
    with pytest.raises(lf.LfbpError):
        lf.compute_Ht_batched([a, a.clone()], outs=[a.clone(), a])   # output 1 is input 0


def test_sixteen_set_table_full_size():
    """The 16-set batch at full size (25.9 GB in, 25.9 GB out): sampled oracle
    check per set, equality with 16 plain launches, and reversibility."""
    dHs, shapes = [], []
    for w in lfsynth.BATCHED_SETS:
        dHs.append(to_dev(lfsynth.bits(w.shape, w.seed, np.float32)))
        shapes.append(w.shape)
    outs = lf.compute_Ht_batched(dHs)
    torch.cuda.synchronize()
    for i, (w, o) in enumerate(zip(lfsynth.BATCHED_SETS, outs)):
        H = lfsynth.bits(w.shape, w.seed, np.float32)
        idx = sample_indices(H.size, 200_000, i)
        got = o.view(-1)[torch.from_numpy(idx).to(DEV)].cpu().numpy()
        assert_same_bits(got, oracle.Ht_at(H, idx), f"set {i} {w.shape}")
        del H
    plain = torch.empty_like(outs[0])
    for i, (h, o) in enumerate(zip(dHs, outs)):
        plain = torch.empty_like(h)
        lf.compute_Ht_into(h, plain)
        assert gpu_equal_bits(plain, o), f"set {i}: batched != plain"
    del plain
    back = lf.compute_Ht_batched(outs)
    for i, (h, b) in enumerate(zip(dHs, back)):
        assert gpu_equal_bits(h, b), f"set {i} not reversible"


@pytest.mark.parametrize("n", [17, 40])
def test_batch_beyond_inline_descriptors(n):
    """More problems than travel in the kernel arguments: the device table path."""
    shapes = mixed_shapes(11 + n, n)
    Hs = [lfsynth.bits(s, 7 * i + 1, np.float32) for i, s in enumerate(shapes)]
    dHs = [to_dev(H) for H in Hs]
    for cfg in (None, {"variant": lf.GATHER_WIDE, "persistent": 2}, {"variant": lf.GATHER_STAGED},
                {"variant": lf.GATHER_DIRECT, "persistent": 1, "grid": 9},
                {"variant": lf.GATHER_WIDE, "persistent": 2, "schedule": 2},
                {"variant": lf.GATHER_WIDE, "persistent": 1, "schedule": 2, "grid": 24}):
        outs = lf.compute_Ht_batched(dHs, config=cfg)
        torch.cuda.synchronize()
        for i, (o, H) in enumerate(zip(outs, Hs)):
            assert_same_bits(o.cpu().numpy(), oracle.Ht_rows(H), f"{n} problems, set {i} {cfg}")


def test_small_set_batch_full_compare():
    """The 64-set batch of small PSFs (launch overhead comparable with the
    work): every set against the oracle, whole arrays, in one launch."""
    Hs = [lfsynth.make_H(w)[0] for w in lfsynth.SMALL_SETS]
    dHs = [to_dev(H) for H in Hs]
    outs = lf.compute_Ht_batched(dHs)
    torch.cuda.synchronize()
    for w, o, H in zip(lfsynth.SMALL_SETS, outs, Hs):
        assert_same_bits(o.cpu().numpy(), oracle.Ht_rows(H), f"{w.name} {w.shape}")
    # the prepared form (direct launch, then graph replay), called again after
    # the PSFs are refreshed in place
    for rep, prepared in enumerate((lf.BatchedHt(dHs), lf.BatchedHt(dHs, use_graph=True))):
        new = [lfsynth.bits(w.shape, 50 * rep + i, np.float32) for i, w in enumerate(lfsynth.SMALL_SETS)]
        for d, h in zip(dHs, new):
            d.copy_(torch.from_numpy(h))
        got = prepared()
        torch.cuda.synchronize()
        for i, (o, h) in enumerate(zip(got, new)):
            assert_same_bits(o.cpu().numpy(), oracle.Ht_rows(h), f"prepared call {rep}, set {i}")


def test_plan_cache_stays_bounded():
    """100 batched calls, each with fresh output tensors (a new pointer table,
    so a new plan each time; 17 problems, so each plan holds a device
    descriptor table): the number of plans the library holds stays at its
    bound, device memory stays flat once the cache is full, and every result
    is still the oracle's."""
    lf.release_plans()
    shapes = mixed_shapes(77, 17)
    Hs = [lfsynth.bits(s, 3 * i + 2, np.float32) for i, s in enumerate(shapes)]
    refs = [oracle.Ht_rows(H) for H in Hs]
    dHs = [to_dev(H) for H in Hs]
    all_outs = [[torch.empty_like(h) for h in dHs] for _ in range(100)]   # distinct pointers every call
    torch.cuda.synchronize()
    free_at = {}
    for k, outs in enumerate(all_outs):
        lf.compute_Ht_batched(dHs, outs)
        if k in (40, 99):
            torch.cuda.synchronize()
            free_at[k] = torch.cuda.mem_get_info()[0]
    torch.cuda.synchronize()
    lf.compute_Ht_batched(dHs, all_outs[-1])          # a known table: reaps finished retired plans
    assert lf.plan_count() <= 32, lf.plan_count()
    assert free_at[99] >= free_at[40] - (64 << 20), (free_at[40] - free_at[99]) / 2 ** 20
    for k in (0, 57, 99):
        for i, (o, r) in enumerate(zip(all_outs[k], refs)):
            assert_same_bits(o.cpu().numpy(), r, f"call {k} set {i}")
    lf.release_plans()
    assert lf.plan_count() == 0


def test_new_table_used_from_a_second_stream_at_once():
    """A plan made by a call on one stream (its device table written by
    kernels on that stream) and used at once, with no synchronisation, by a
    call on another stream: the second launch waits for the table."""
    lf.release_plans()
    shapes = mixed_shapes(91, 24)
    Hs = [lfsynth.bits(s, 11 * i + 5, np.float32) for i, s in enumerate(shapes)]
    dHs = [to_dev(H) for H in Hs]
    outs_a = [torch.empty_like(h) for h in dHs]
    outs_b = [torch.empty_like(h) for h in dHs]
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    busy = torch.empty(1 << 26, device=DEV)
    with torch.cuda.stream(sa):
        busy.normal_()                                  # keeps stream a busy before the table is written
        lf.compute_Ht_batched(dHs, outs_a)
    with torch.cuda.stream(sb):
        lf.compute_Ht_batched(dHs, outs_a)              # same table, same plan, other stream
        lf.compute_Ht_batched(dHs, outs_b)
    torch.cuda.synchronize()
    for i, H in enumerate(Hs):
        ref = oracle.Ht_rows(H)
        assert_same_bits(outs_a[i].cpu().numpy(), ref, f"set {i}")
        assert_same_bits(outs_b[i].cpu().numpy(), ref, f"set {i}, second table")
    lf.release_plans()


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")  # the first capture is refused on purpose
def test_table_of_many_problems_first_made_under_capture():
    """A 20-problem table submitted first inside a caller's stream capture
    needs a device table, which cannot be allocated there: the call returns
    ECAPTURE before any HIP call and the capture stays valid.  Submitted once
    outside, the same table is then captured, and every replay gives the
    oracle's H'."""
    from paper_2003_09133_amd import _abi
    lf.release_plans()
    shapes = mixed_shapes(5, 20)
    dHs = [torch.empty(s, dtype=torch.float32, device=DEV) for s in shapes]
    outs = [torch.empty_like(h) for h in dHs]
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        with pytest.raises(lf.LfbpError) as err:
            lf.compute_Ht_batched(dHs, outs)
    assert err.value.status == _abi.ECAPTURE
    assert lf.plan_count() == 0
    lf.compute_Ht_batched(dHs, outs)                    # makes the plan
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        lf.compute_Ht_batched(dHs, outs)
    for rep in range(3):
        hs = [lfsynth.bits(s, 70 * rep + i, np.float32) for i, s in enumerate(shapes)]
        for d, h in zip(dHs, hs):
            d.copy_(torch.from_numpy(h))
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for i, (o, h) in enumerate(zip(outs, hs)):
            assert_same_bits(o.cpu().numpy(), oracle.Ht_rows(h), f"replay {rep} set {i}")
    del graph
    lf.release_plans()
