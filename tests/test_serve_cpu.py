"""CPU checks of the serving loop's host logic: latency percentiles on a
synthetic clock, in-order admission under the HBM budget, the trace recipe."""
import numpy as np

from paper_2604_00567_amd import inputs
from paper_2604_00567_amd import binding
from paper_2604_00567_amd.serve import ELEM_BYTES, admit_step, is_split, latency_summary, request_bytes


def test_latency_summary_synthetic_clock():
    lat = np.arange(1, 1001) * 1e-3          # 1 ms .. 1000 ms
    s = latency_summary(lat)
    assert abs(s["p50_ms"] - 500.5) < 1e-9
    assert abs(s["p99_ms"] - 990.01) < 1e-9
    assert s["max_ms"] == 1000.0 and s["count"] == 1000
    assert latency_summary(np.array([]))["count"] == 0


def _trace(k, seed):
    return inputs.poisson_trace(20000.0, k / 20000.0, seed)


def test_admission_respects_budget_and_order():
    tr = _trace(2000, 3)
    total = tr["t"].size
    nb = [request_bytes(int(n), int(b), str(d)) for n, b, d in zip(tr["n"], tr["batch"], tr["dtype"])]
    pending = list(range(total))
    budget = 512 << 20

    def fits(plan, n, b, dt):
        return plan[dt][0] + n * b <= (256 << 20) // ELEM_BYTES[dt]

    head, inflight, seen = 0, 0, []
    steps = 0
    while head < total:
        take, head2, inflight2 = admit_step(pending, head, tr, inflight, budget, fits, 64, nb)
        if not take:                             # nothing fits: everything in flight completes
            inflight = 0
            continue
        assert take == pending[head:head2]       # arrival order, no skipping
        # in flight grows by the requests' bytes; each was admitted only with
        # room for its workspace too (the slot's own arena holds it)
        assert inflight2 == inflight + sum(nb[r] for r in take)
        room = inflight
        for r in take:
            n, dt = int(tr["n"][r]), str(tr["dtype"][r])
            ws = n * int(tr["batch"][r]) * ELEM_BYTES[dt] if is_split(n, dt) else 0
            assert room + nb[r] + ws <= budget
            room += nb[r]
        seen += take
        head, inflight = head2, inflight2
        steps += 1
        if steps % 3 == 0:
            inflight = 0                         # completions free the budget
    assert seen == list(range(total))


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
