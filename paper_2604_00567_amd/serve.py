"""Continuous-batching FFT serving on one GPU (the loops run natively in the
library: ``fft_serve_run``).

Requests (N = 2^k up to 2^18 points, a batch of such transforms, binary16 or
binary32) arrive over time.  The continuous loop admits them in arrival order
whenever one of K slots is free and they fit the HBM budget, generates their
data on the device, and launches one step per precision on the slot's stream
(the serving-slot batch kernels, or for a step of one or two requests one
cached-plan launch each; split-size transforms through their cached two-pass
plans); K slots run on K streams, so a step
admitted while earlier steps are still on the GPU overlaps with them.
``run_per_request`` replays the same trace with one cached-plan launch per
request, the form the continuous loop is compared with.  Latency of a request
= the host time at which its completion is observed minus its arrival time.

This module turns the native results into latency percentiles and, when asked
(``keep_io``), into per-request input and output tensors for checks: the
outputs are copied by the loop itself, the inputs regenerated with the loop's
own generator (``fft_serve_fill``), which keys each request's data by its
position among the requests of its precision.
"""
from __future__ import annotations

import numpy as np

from . import binding

ELEM_BYTES = {"f16": 4, "f32": 8}
# log2 of the largest transform that runs whole (binary16: the 2^15 and 2^16
# list kernels; binary32: whole-transform work items); larger ones take the
# column/row split and a workspace slice
MAX_WHOLE_LOG = {"f16": 16, "f32": 14}


def is_split(n: int, dtype: str) -> bool:
    return n > (1 << MAX_WHOLE_LOG[dtype])


def latency_summary(latency_s: np.ndarray) -> dict:
    """p50 / p99 / mean / max of latencies given in seconds, reported in ms."""
    lat = np.asarray(latency_s, dtype=np.float64)
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "mean_ms": None, "max_ms": None, "count": 0}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3),
            "count": int(lat.size)}


def request_bytes(n: int, batch: int, dtype: str) -> int:
    """Algorithmic bytes of a request: one read and one write of its data."""
    return 2 * n * batch * ELEM_BYTES[dtype]


def generator_offsets(trace) -> np.ndarray:
    """Each request's first element in its precision's generator stream: the
    elements of the earlier requests of that precision, in arrival order."""
    first = np.zeros(len(trace["n"]), np.int64)
    pos = {"f16": 0, "f32": 0}
    for r, (n, b, d) in enumerate(zip(trace["n"], trace["batch"], trace["dtype"])):
        d = str(d)
        first[r] = pos[d]
        pos[d] += int(n) * int(b)
    return first


def _io_buffers(trace):
    """A device buffer for every request's output and each one's byte offset."""
    import torch
    sizes = [int(n) * int(b) * ELEM_BYTES[str(d)] for n, b, d in zip(trace["n"], trace["batch"], trace["dtype"])]
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if sizes else np.zeros(0, np.int64)
    buf = torch.empty(max(1, int(np.sum(sizes))), dtype=torch.uint8, device="cuda")
    return buf, off, sizes


def _views(trace, buf, off, sizes, seed):
    """(inputs, outputs): per request, its regenerated input and its output."""
    import torch
    tdt = {"f16": torch.float16, "f32": torch.float32}
    first = generator_offsets(trace)
    ins, outs = {}, {}
    for r, (n, b, d) in enumerate(zip(trace["n"], trace["batch"], trace["dtype"])):
        d = str(d)
        outs[r] = buf[int(off[r]):int(off[r]) + sizes[r]].view(tdt[d])
        x = torch.empty(2 * int(n) * int(b), dtype=tdt[d], device="cuda")
        binding.fft_serve_fill(d, x.data_ptr(), int(n) * int(b), int(first[r]), seed)
        ins[r] = x
    torch.cuda.synchronize()
    return ins, outs


def _summary(trace, done, st, extra) -> dict:
    t = np.asarray(trace["t"], np.float64)
    nb = sum(request_bytes(int(n), int(b), str(d)) for n, b, d in zip(trace["n"], trace["batch"], trace["dtype"]))
    out = latency_summary(done - t)
    wall = float(st.wall_s) if st.wall_s > 0 else float("nan")
    out.update({"requests": int(t.size), "gbs": float(nb / wall / 1e9), "wall_s": wall,
                "max_inflight_bytes": int(st.max_inflight_bytes)})
    out.update(extra)
    return out


class Server:
    """K-slot continuous-batching server (``fft_serve_run``, continuous mode).
    ``budget_bytes`` caps the request data (plus large-transform workspace)
    admitted but not yet completed.  A step of at most ``direct_max``
    requests launches each through a cached plan (two-pass plans on a
    workspace of the slot); larger steps run the slot's batch kernels.  With
    ``split_direct`` the split-size transforms (column/row schedule) of every
    step take their cached two-pass plans after the step's other requests,
    which complete on an event of their own.  All forms compute every
    transform with the same butterflies and table, bit for bit."""

    def __init__(self, slots: int = 4, budget_bytes: int = 64 << 30, slot_bytes: int = 1 << 30,
                 kind: str = "dual_select", max_transforms: int = 1 << 15,
                 max_large: int = 1 << 12, max_items: int = 1 << 18, seed: int = 0,
                 keep_io: bool = False, direct_max: int = 2, split_direct: bool = True):
        self.slots, self.budget, self.slot_bytes = int(slots), int(budget_bytes), int(slot_bytes)
        self.kind, self.seed, self.keep_io, self.direct_max = kind, int(seed), keep_io, int(direct_max)
        self.split_direct = bool(split_direct)
        self.max_transforms, self.max_large, self.max_items = int(max_transforms), int(max_large), int(max_items)
        self.inputs, self.outputs = {}, {}

    def config(self, max_step_requests: int = 256) -> binding.ServeConfig:
        return binding.ServeConfig(
            mode=binding.FFT_SERVE_CONTINUOUS, slots=self.slots, kind=binding.KINDS[self.kind],
            direct_max=self.direct_max, max_step_requests=int(max_step_requests), max_large=self.max_large,
            max_transforms=self.max_transforms, max_items=self.max_items, budget_bytes=self.budget,
            slot_bytes=self.slot_bytes, seed=self.seed, split_direct=int(self.split_direct))

    def run(self, trace: dict, max_step_requests: int = 256) -> dict:
        cfg = self.config(max_step_requests)
        if self.keep_io:
            buf, off, sizes = _io_buffers(trace)
            done, st = binding.fft_serve_run(cfg, trace, buf.data_ptr(), off)
            self.inputs, self.outputs = _views(trace, buf, off, sizes, self.seed)
        else:
            done, st = binding.fft_serve_run(cfg, trace)
        return _summary(trace, done, st, {
            "steps": int(st.steps), "mean_requests_per_step": float(st.mean_requests_per_step),
            "budget_bytes": self.budget, "max_concurrent_steps": int(st.max_concurrent),
            "slots": self.slots, "direct_steps": int(st.direct_steps), "direct_max": self.direct_max,
            "split_direct": self.split_direct})

    def close(self):
        """Nothing to release: each run allocates and frees its own slots.  The
        kept inputs and outputs stay until the next run."""


def run_per_request(trace: dict, streams: int = 4, kind: str = "dual_select", seed: int = 0,
                    budget_bytes: int = 64 << 30, keep_io: dict = None,
                    ring_bytes: int = 1 << 30) -> dict:
    """Same trace, one launch per request (``fft_serve_run``, per-request
    mode): cached plans per shape and stream (a two-pass plan owns one
    workspace and must not run on two streams at once), round-robin over
    `streams` streams, admitted in arrival order under the same HBM budget.
    ``keep_io``: a dict that receives {rid: (input, output)} device tensors."""
    cfg = binding.ServeConfig(
        mode=binding.FFT_SERVE_PER_REQUEST, slots=int(streams), kind=binding.KINDS[kind], direct_max=0,
        max_step_requests=1, max_large=0, max_transforms=1, max_items=1, budget_bytes=int(budget_bytes),
        slot_bytes=int(ring_bytes), seed=int(seed))
    if keep_io is not None:
        buf, off, sizes = _io_buffers(trace)
        done, st = binding.fft_serve_run(cfg, trace, buf.data_ptr(), off)
        ins, outs = _views(trace, buf, off, sizes, seed)
        for r in ins:
            keep_io[r] = (ins[r], outs[r])
    else:
        done, st = binding.fft_serve_run(cfg, trace)
    return _summary(trace, done, st, {"launches": int(np.asarray(trace["t"]).size), "streams": int(streams),
                                      "budget_bytes": int(budget_bytes)})
