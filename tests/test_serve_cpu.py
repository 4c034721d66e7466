"""CPU checks of the serving loop's host logic: latency percentiles on a
synthetic clock, in-order admission under the HBM budget, the trace recipe."""
import numpy as np

from paper_2604_00567_amd import inputs
from paper_2604_00567_amd import binding
from paper_2604_00567_amd.serve import ELEM_BYTES, generator_offsets, is_split, latency_summary, request_bytes


def test_latency_summary_synthetic_clock():
    lat = np.arange(1, 1001) * 1e-3          # 1 ms .. 1000 ms
    s = latency_summary(lat)
    assert abs(s["p50_ms"] - 500.5) < 1e-9
    assert abs(s["p99_ms"] - 990.01) < 1e-9
    assert s["max_ms"] == 1000.0 and s["count"] == 1000
    assert latency_summary(np.array([]))["count"] == 0


def _trace(k, seed):
    return inputs.poisson_trace(20000.0, k / 20000.0, seed)


def _cfg(budget, slot_bytes=256 << 20, max_step=64):
    return binding.ServeConfig(mode=binding.FFT_SERVE_CONTINUOUS, slots=4, kind=0, direct_max=2,
                               max_step_requests=max_step, max_large=1 << 12, max_transforms=1 << 15,
                               max_items=1 << 18, budget_bytes=budget, slot_bytes=slot_bytes, seed=0)


def test_admission_respects_budget_and_order():
    # the library's own admission rule (the continuous loop calls the same code)
    tr = _trace(2000, 3)
    total = tr["t"].size
    nb = [request_bytes(int(n), int(b), str(d)) for n, b, d in zip(tr["n"], tr["batch"], tr["dtype"])]
    budget = 512 << 20
    cfg = _cfg(budget)
    head, inflight, seen = 0, 0, []
    steps = 0
    while head < total:
        take, inflight2 = binding.fft_serve_admit(tr, head, inflight, cfg)
        if not take:                             # nothing fits: everything in flight completes
            assert inflight > 0
            inflight = 0
            continue
        assert take == list(range(head, head + len(take)))     # arrival order, no skipping
        assert len(take) <= cfg.max_step_requests
        # in flight grows by the requests' bytes; each was admitted only with
        # room for its workspace too
        assert inflight2 == inflight + sum(nb[r] for r in take)
        room = inflight
        used = {"f16": 0, "f32": 0}
        for r in take:
            n, dt = int(tr["n"][r]), str(tr["dtype"][r])
            ws = n * int(tr["batch"][r]) * ELEM_BYTES[dt] if is_split(n, dt) else 0
            assert room + nb[r] + ws <= budget
            room += nb[r]
            used[dt] += n * int(tr["batch"][r]) * ELEM_BYTES[dt]
        assert max(used.values()) <= cfg.slot_bytes              # the slot's arena per precision
        # the next request did not fit (or the step was full)
        if head + len(take) < total and len(take) < cfg.max_step_requests:
            r = head + len(take)
            n, dt = int(tr["n"][r]), str(tr["dtype"][r])
            ws = n * int(tr["batch"][r]) * ELEM_BYTES[dt] if is_split(n, dt) else 0
            over_budget = inflight2 + nb[r] + ws > budget
            over_slot = used[dt] + n * int(tr["batch"][r]) * ELEM_BYTES[dt] > cfg.slot_bytes
            assert over_budget or over_slot
        seen += take
        head, inflight = head + len(take), inflight2
        steps += 1
        if steps % 3 == 0:
            inflight = 0                         # completions free the budget
    assert seen == list(range(total))


def test_admission_whole_transform_capacity():
    # many whole-size requests: a step stops at the slot's transform capacity
    k = 50
    tr = {"n": np.full(k, 256, np.int64), "batch": np.full(k, 64, np.int64), "dtype": np.array(["f16"] * k)}
    cfg = _cfg(1 << 40)
    cfg.max_transforms = 64 * 7 + 10
    take, _ = binding.fft_serve_admit(tr, 0, 0, cfg)
    assert take == list(range(7))


def test_trace_recipe():
    tr = inputs.poisson_trace(20000.0, 1.0, 11)
    k = tr["t"].size
    assert 19000 < k < 21000                                # Poisson count around 20k
    assert np.all(np.diff(tr["t"]) > 0)
    logn = np.log2(tr["n"]).astype(int)
    assert logn.min() >= 8 and logn.max() <= 18
    assert tr["batch"].min() >= 1 and tr["batch"].max() <= 64
    assert 0.72 < np.mean(tr["dtype"] == "f16") < 0.78


def test_split_rule_matches_the_library():
    """The serving loop reserves workspace exactly for the transforms the
    library splits into column and row items (its work list's workspace)."""
    for dt in ("f16", "f32"):
        for m in range(1, 19):
            n = 1 << m
            _, _, _, _, ws = binding.fft_batch_work_list([n, n], dt)
            assert (ws > 0) == is_split(n, dt), (dt, m)
            assert ws == (2 * n if is_split(n, dt) else 0)


def test_generator_offsets():
    tr = {"n": np.array([4, 8, 16, 2]), "batch": np.array([1, 2, 1, 3]), "dtype": np.array(["f16", "f32", "f16", "f32"])}
    assert generator_offsets(tr).tolist() == [0, 0, 4, 16]


def _items(sizes, dt):
    """Work items of the slot kernels for these transforms (the library's own list)."""
    return binding.fft_batch_work_list(sizes, dt)[0].shape[0]


def test_admission_work_item_capacity_whole_sizes():
    # 256-point transforms share items of several units each: a step stops
    # exactly where one more transform would open an item beyond max_items
    k = 200
    tr = {"n": np.full(k, 256, np.int64), "batch": np.ones(k, np.int64), "dtype": np.array(["f16"] * k)}
    cfg = _cfg(1 << 40, max_step=k)
    cfg.max_items = 1
    take, _ = binding.fft_serve_admit(tr, 0, 0, cfg)
    assert 1 < len(take) < k
    assert _items([256] * len(take), "f16") == 1
    assert _items([256] * (len(take) + 1), "f16") == 2


def test_admission_work_item_capacity_split_sizes():
    # binary32 2^15 transforms take the column/row split: each adds its column
    # and row items, unless split transforms run through their plans
    k = 40
    n = 1 << 15
    tr = {"n": np.full(k, n, np.int64), "batch": np.full(k, 4, np.int64), "dtype": np.array(["f32"] * k)}
    per = _items([n], "f32")
    assert per > 1
    cfg = _cfg(1 << 40, slot_bytes=1 << 30, max_step=k)
    cfg.max_items = 10 * per
    take, _ = binding.fft_serve_admit(tr, 0, 0, cfg)
    assert len(take) == 2                                 # 8 transforms; a third request makes 12
    assert _items([n] * 8, "f32") <= cfg.max_items < _items([n] * 12, "f32")
    cfg.split_direct = 1
    take, _ = binding.fft_serve_admit(tr, 0, 0, cfg)
    assert len(take) > 2


def test_admission_rejects_bad_requests():
    import pytest
    cfg = _cfg(1 << 40)
    for n, b, dt in ((1 << 19, 1, "f16"), (3, 1, "f16"), (256, 0, "f32")):
        tr = {"n": np.array([n]), "batch": np.array([b]), "dtype": np.array([dt])}
        with pytest.raises(RuntimeError):
            binding.fft_serve_admit(tr, 0, 0, cfg)
