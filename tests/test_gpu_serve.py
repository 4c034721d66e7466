"""GPU tests of the continuous-batching serving loop: every checked request's
result is the same alone (a regular plan on the same input) as in the mix,
steps batch several requests and overlap on the device, and admission keeps
in-flight bytes under the budget."""
import numpy as np
import pytest

import oracle
from paper_2604_00567_amd import binding, inputs
from paper_2604_00567_amd.serve import Server, run_per_request
from tests.gpu_util import mismatches

pytestmark = pytest.mark.gpu


def small_trace(k, seed, rate=200000.0, log_hi=14, batch_hi=8):
    tr = inputs.poisson_trace(rate, k / rate, seed, log_lo=8, log_hi=log_hi, batch_hi=batch_hi)
    return tr


def plan_alone(x, n, b, dt):
    import torch
    y = torch.empty_like(x)
    p = binding.Plan(n, b, dt, "dual_select")
    try:
        p.execute(x.view(b, n, 2), y.view(b, n, 2))
        torch.cuda.synchronize()
    finally:
        p.close()
    return y


def test_results_alone_equal_results_in_mix():
    import torch
    tr = small_trace(400, 21, log_hi=16)
    srv = Server(slots=3, slot_bytes=256 << 20, keep_io=True, seed=5)
    try:
        stats = srv.run(tr, max_step_requests=32)
        torch.cuda.synchronize()
    finally:
        srv.close()
    assert stats["requests"] == tr["t"].size
    assert stats["mean_requests_per_step"] > 1.0           # steps batch requests
    assert stats["max_concurrent_steps"] >= 2               # steps overlap on the device
    rng = np.random.default_rng(0)
    pick = rng.choice(tr["t"].size, 40, replace=False)
    for rid in pick:
        n, b, dt = int(tr["n"][rid]), int(tr["batch"][rid]), str(tr["dtype"][rid])
        x = srv.inputs[rid].reshape(b, n, 2)
        y_mix = srv.outputs[rid].reshape(b, n, 2)
        y_alone = torch.empty_like(x)
        p = binding.Plan(n, b, dt, "dual_select")
        p.execute(x, y_alone)
        torch.cuda.synchronize()
        p.close()
        assert mismatches(y_mix.cpu().numpy(), y_alone.cpu().numpy()) == 0, (rid, n, b, dt)
    # and a few against the oracle's emulation
    for rid in pick[:6]:
        n, b, dt = int(tr["n"][rid]), int(tr["batch"][rid]), str(tr["dtype"][rid])
        x = srv.inputs[rid].reshape(b, n, 2).cpu().numpy()
        y = srv.outputs[rid].reshape(b, n, 2).cpu().numpy()
        assert mismatches(y, oracle.emulate(x, "dual_select", dt)) == 0


def test_small_steps_run_through_plans_with_the_same_results():
    """At a low arrival rate most steps hold one or two requests and take the
    direct form (one plan launch per request); a request's data depend only on
    its position in the trace, so the direct form, the batch-kernel form and
    one launch per request give the same outputs bit for bit, and they equal
    the oracle's."""
    import torch
    tr = small_trace(120, 24, rate=4000.0, log_hi=16)
    outs = {}
    for direct_max in (2, 0):
        srv = Server(slots=2, slot_bytes=64 << 20, keep_io=True, seed=7, direct_max=direct_max)
        try:
            stats = srv.run(tr)
            torch.cuda.synchronize()
        finally:
            ins, res = dict(srv.inputs), dict(srv.outputs)
            srv.close()
        assert stats["requests"] == tr["t"].size
        if direct_max:
            assert stats["direct_steps"] > 0
        else:
            assert stats["direct_steps"] == 0
        outs[direct_max] = (ins, res)
    io = {}
    run_per_request(tr, streams=2, seed=7, keep_io=io)
    torch.cuda.synchronize()
    for rid in range(tr["t"].size):
        a = outs[2][1][rid].cpu().numpy()
        assert mismatches(a, outs[0][1][rid].cpu().numpy()) == 0, rid
        assert mismatches(a, io[rid][1].cpu().numpy()) == 0, rid
        assert mismatches(outs[2][0][rid].cpu().numpy(), io[rid][0].cpu().numpy()) == 0, rid
    ins, res = outs[2]
    for rid in range(0, tr["t"].size, 7):
        n, b, dt = int(tr["n"][rid]), int(tr["batch"][rid]), str(tr["dtype"][rid])
        y_alone = plan_alone(ins[rid], n, b, dt)
        assert mismatches(res[rid].cpu().numpy(), y_alone.cpu().numpy()) == 0
    for rid in range(0, tr["t"].size, 30):
        n, b, dt = int(tr["n"][rid]), int(tr["batch"][rid]), str(tr["dtype"][rid])
        x = ins[rid].reshape(b, n, 2).cpu().numpy()
        assert mismatches(res[rid].reshape(b, n, 2).cpu().numpy(), oracle.emulate(x, "dual_select", dt)) == 0


def test_payload_generator():
    """The serving payload generator: deterministic, keyed by element index (a
    slice of a longer draw equals the draw of that slice), N(0, 1) moments,
    different for the two precisions' streams and for another seed."""
    import torch
    m = 1 << 20
    a = torch.empty(2 * m, dtype=torch.float32, device="cuda")
    b = torch.empty(2 * 1000, dtype=torch.float32, device="cuda")
    c = torch.empty(2 * m, dtype=torch.float32, device="cuda")
    h = torch.empty(2 * m, dtype=torch.float16, device="cuda")
    binding.fft_serve_fill("f32", a.data_ptr(), m, 0, 11)
    binding.fft_serve_fill("f32", b.data_ptr(), 1000, 5000, 11)
    binding.fft_serve_fill("f32", c.data_ptr(), m, 0, 12)
    binding.fft_serve_fill("f16", h.data_ptr(), m, 0, 11)
    torch.cuda.synchronize()
    av = a.cpu().numpy()
    assert np.array_equal(av[10000:12000], b.cpu().numpy())
    assert abs(av.mean()) < 5e-3 and abs(av.var() - 1.0) < 5e-3
    assert abs(np.mean(av ** 4) - 3.0) < 0.05                      # normal kurtosis
    assert not np.array_equal(av, c.cpu().numpy())
    hv = h.cpu().numpy().astype(np.float64)
    assert np.isfinite(hv).all() and abs(hv.var() - 1.0) < 5e-3
    assert np.mean(np.abs(hv - av) < 1e-2) < 0.01                  # another stream, not a rounded copy


def test_budget_is_respected():
    tr = small_trace(300, 22)
    budget = 48 << 20
    srv = Server(slots=4, budget_bytes=budget, slot_bytes=64 << 20, seed=6)
    try:
        stats = srv.run(tr)
    finally:
        srv.close()
    assert stats["requests"] == tr["t"].size
    assert 0 < stats["max_inflight_bytes"] <= budget


def test_per_request_baseline_runs():
    tr = small_trace(200, 23, rate=20000.0)
    stats = run_per_request(tr, streams=2)
    assert stats["requests"] == tr["t"].size and stats["p99_ms"] >= stats["p50_ms"] > 0


def test_large_requests_alone_equal_results_in_mix():
    """The serving workload's full size range (N up to 2^18, batch up to 64):
    the column/row split of binary16 2^17-2^18 and binary32 2^15-2^18 runs in
    the slots' batch kernels beside whole transforms; every split-size request
    and a sample of the others equal a regular plan on the same input, and a
    few equal the oracle's emulation.  Running the split transforms through
    their two-pass plans instead gives every request the same output."""
    import torch
    tr = small_trace(160, 31, rate=400000.0, log_hi=18, batch_hi=64)
    srv = Server(slots=3, slot_bytes=512 << 20, keep_io=True, seed=9, split_direct=False)
    try:
        stats = srv.run(tr, max_step_requests=32)
        torch.cuda.synchronize()
    finally:
        srv.close()
    assert stats["requests"] == tr["t"].size
    assert stats["mean_requests_per_step"] > 1.0
    # split transforms through their two-pass plans, the rest of each step
    # completing on its own event: the same outputs bit for bit
    srv2 = Server(slots=3, slot_bytes=512 << 20, keep_io=True, seed=9, split_direct=True)
    stats2 = srv2.run(tr, max_step_requests=32)
    torch.cuda.synchronize()
    assert stats2["requests"] == tr["t"].size and stats2["mean_requests_per_step"] > 1.0
    for rid in range(tr["t"].size):
        assert mismatches(srv2.outputs[rid].cpu().numpy(), srv.outputs[rid].cpu().numpy()) == 0, rid
    del srv2
    n_all, b_all, d_all = tr["n"], tr["batch"], tr["dtype"]
    split_ids = [r for r in range(tr["t"].size)
                 if n_all[r] > (1 << (16 if d_all[r] == "f16" else 14))]
    assert any(d_all[r] == "f16" for r in split_ids) and any(d_all[r] == "f32" for r in split_ids)
    rng = np.random.default_rng(1)
    others = [r for r in range(tr["t"].size) if r not in split_ids]
    check = split_ids[:24] + list(rng.choice(others, 16, replace=False))
    for rid in check:
        n, b, dt = int(n_all[rid]), int(b_all[rid]), str(d_all[rid])
        y_alone = plan_alone(srv.inputs[rid], n, b, dt)
        assert mismatches(srv.outputs[rid].cpu().numpy(), y_alone.cpu().numpy()) == 0, (rid, n, b, dt)
    small_split = [r for r in split_ids if n_all[r] * b_all[r] <= (1 << 21)][:3]
    for rid in small_split + check[-3:]:
        n, b, dt = int(n_all[rid]), int(b_all[rid]), str(d_all[rid])
        x = srv.inputs[rid].reshape(b, n, 2).cpu().numpy()
        y = srv.outputs[rid].reshape(b, n, 2).cpu().numpy()
        assert mismatches(y, oracle.emulate(x, "dual_select", dt)) == 0, (rid, n, b, dt)


def test_per_request_baseline_two_pass_plans_per_stream():
    """One launch per request with many same-shape two-pass requests in flight
    on several streams at once: each stream's plan has its own workspace, so
    every result equals the same plan run alone."""
    import torch
    k = 48
    tr = {"t": np.linspace(0.0, 1e-4, k), "n": np.full(k, 1 << 17, np.int64),
          "batch": np.full(k, 4, np.int64),
          "dtype": np.array(["f16", "f32"] * (k // 2))}
    io = {}
    stats = run_per_request(tr, streams=4, seed=3, keep_io=io)
    torch.cuda.synchronize()
    assert stats["requests"] == k and len(io) == k
    for rid, (x, y) in io.items():
        n, b, dt = int(tr["n"][rid]), int(tr["batch"][rid]), str(tr["dtype"][rid])
        y_alone = plan_alone(x, n, b, dt)
        assert mismatches(y.cpu().numpy(), y_alone.cpu().numpy()) == 0, (rid, dt)
