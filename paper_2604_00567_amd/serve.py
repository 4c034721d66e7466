"""Continuous-batching FFT serving loop on one GPU.

Requests (N = 2^k up to 2^18 points, a batch of such transforms, binary16 or
binary32) arrive over time.  The loop admits them in arrival order whenever a
slot is free and they fit the HBM budget, packs the requests of one
scheduling step into the slot's device arena (one region per precision), and
launches one persistent-kernel step per precision on the slot's stream
(``fft_serve_slot_launch``).  K slots run on K streams, so a step admitted
while earlier steps are still on the GPU overlaps with them.  Plans and
twiddle tables stay resident in the slots for the whole run.  Latency of a
request = the host time at which its step's completion is observed minus its
arrival time.

``run_per_request`` replays the same trace with one launch per request
through cached regular plans, the form the continuous loop is compared with.
Payloads are generated on the GPU (torch's N(0,1) generator), so no request
data crosses PCIe.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding

ELEM_BYTES = {"f16": 4, "f32": 8}
TORCH_DTYPE = {"f16": torch.float16, "f32": torch.float32}
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


def admit_step(pending, head, trace, inflight, budget, fits, max_step_requests, nbytes):
    """Takes requests from pending[head:] in arrival order while each fits the
    HBM budget (request bytes plus large-transform workspace on top of what is
    in flight) and the step's capacities (``fits(plan, n, b, dtype)``).  Stops
    at the first request that does not fit, so admission stays in order.
    Returns (taken ids, new head, new in-flight bytes)."""
    plan = {"f16": [0, 0, 0, 0], "f32": [0, 0, 0, 0]}
    take = []
    while head < len(pending) and len(take) < max_step_requests:
        rid = pending[head]
        n, b, dt = int(trace["n"][rid]), int(trace["batch"][rid]), str(trace["dtype"][rid])
        ws = n * b * ELEM_BYTES[dt] if is_split(n, dt) else 0
        if inflight + nbytes[rid] + ws > budget or not fits(plan, n, b, dt):
            break
        p = plan[dt]
        p[0] += n * b
        if is_split(n, dt):
            p[2] += b
            p[3] += n * b
        else:
            p[1] += b
        take.append(rid)
        inflight += nbytes[rid]
        head += 1
    return take, head, inflight


@dataclass
class _Slot:
    stream: torch.cuda.Stream
    arena: dict
    native: dict
    cap_elems: int
    ws_elems: int
    event: torch.cuda.Event = None
    busy: bool = False
    rids: list = field(default_factory=list)
    bytes: int = 0
    placement: dict = field(default_factory=dict)     # rid -> (dtype, offset, n, batch)


class Server:
    """K-slot continuous-batching server.  ``budget_bytes`` caps the request
    data (plus large-transform workspace) admitted but not yet completed.

    A step of at most ``direct_max`` requests that all run whole (no
    column/row split) launches each request through a cached plan on the
    slot's stream, in place in the slot's arena: for one or two requests that
    is one kernel each, where the batch kernels add a staging copy and a list
    or phase launch.  Larger steps run the batch kernels.  Both forms compute
    every transform with the same butterflies and table, bit for bit."""

    def __init__(self, slots: int = 4, budget_bytes: int = 64 << 30, slot_bytes: int = 1 << 30,
                 kind: str = "dual_select", max_transforms: int = 1 << 15,
                 max_large: int = 1 << 12, max_items: int = 1 << 18, seed: int = 0,
                 keep_io: bool = False, direct_max: int = 2):
        self.budget = int(budget_bytes)
        self.kind = kind
        self.keep_io = keep_io
        self.direct_max = int(direct_max)
        self.plans = {}
        self.direct_steps = 0
        self.gen = torch.Generator(device="cuda")
        self.gen.manual_seed(seed)
        self.slots = []
        for _ in range(slots):
            arena, native = {}, {}
            cap = {}
            for dt in ("f16", "f32"):
                elems = slot_bytes // ELEM_BYTES[dt]
                cap[dt] = elems
                arena[dt] = torch.empty(elems * 2, dtype=TORCH_DTYPE[dt], device="cuda")
                native[dt] = binding.fft_serve_slot_create(dt, kind, max_items, max_transforms,
                                                           max_large, slot_bytes)
            self.slots.append(_Slot(stream=torch.cuda.Stream(), arena=arena, native=native,
                                    cap_elems=cap["f16"], ws_elems=slot_bytes))
        self.max_transforms, self.max_large = max_transforms, max_large
        self.slot_bytes = slot_bytes
        self.inputs, self.outputs = {}, {}

    def close(self):
        for s in self.slots:
            for h in s.native.values():
                binding.fft_serve_slot_destroy(h)
        self.slots = []
        for p in self.plans.values():
            p.close()
        self.plans = {}

    def _plan(self, n, b, dt):
        key = (n, b, dt)
        if key not in self.plans:
            self.plans[key] = binding.Plan(n, b, dt, self.kind)
        return self.plans[key]

    # ------------------------------------------------------------------ steps
    def _fits(self, plan, n, b, dt):
        used, transforms, large, ws = plan[dt]
        elems = n * b
        cap = self.slot_bytes // ELEM_BYTES[dt]
        if used + elems > cap:
            return False
        if is_split(n, dt):
            if large + b > self.max_large or (ws + elems) * ELEM_BYTES[dt] > self.slot_bytes:
                return False
        elif transforms + b > self.max_transforms:
            return False
        return True

    def _launch(self, slot: _Slot, reqs, trace):
        """Packs reqs into the slot's arenas, fills them with N(0,1) data and
        launches one step per precision on the slot's stream."""
        per_dt = {"f16": [], "f32": []}
        plan = {"f16": [0, 0, 0, 0], "f32": [0, 0, 0, 0]}
        slot.placement = {}
        for rid in reqs:
            n, b, dt = int(trace["n"][rid]), int(trace["batch"][rid]), str(trace["dtype"][rid])
            p = plan[dt]
            off = p[0]
            per_dt[dt].append((rid, n, b, off))
            slot.placement[rid] = (dt, off, n, b)
            p[0] += n * b
            if is_split(n, dt):
                p[2] += b
                p[3] += n * b
            else:
                p[1] += b
        direct = len(reqs) <= self.direct_max and not any(
            is_split(n, dt) for dt, lst in per_dt.items() for _, n, _, _ in lst)
        self.direct_steps += int(direct)
        with torch.cuda.stream(slot.stream):
            for dt, lst in per_dt.items():
                if not lst:
                    continue
                used = plan[dt][0]
                region = slot.arena[dt][: used * 2]
                region.normal_(0.0, 1.0, generator=self.gen)
                if self.keep_io:
                    for rid, n, b, off in lst:
                        self.inputs[rid] = region[off * 2:(off + n * b) * 2].clone()
                if direct:
                    for _, n, b, off in lst:
                        view = slot.arena[dt][off * 2:(off + n * b) * 2].view(b, n, 2)
                        self._plan(n, b, dt).execute(view, view, stream=slot.stream)
                    continue
                arr = np.asarray([(n, b, off) for _, n, b, off in lst], dtype=np.int64)
                binding.fft_serve_slot_launch(slot.native[dt], arr[:, 0], arr[:, 1], arr[:, 2],
                                              slot.arena[dt].data_ptr(), slot.stream.cuda_stream)
            slot.event = torch.cuda.Event()
            slot.event.record(slot.stream)
        slot.busy = True
        slot.rids = list(reqs)

    def _complete(self, slot: _Slot):
        if self.keep_io:
            # copies on the slot's stream, ahead of the slot's next step
            with torch.cuda.stream(slot.stream):
                for rid, (dt, off, n, b) in slot.placement.items():
                    self.outputs[rid] = slot.arena[dt][off * 2:(off + n * b) * 2].clone()
        slot.busy = False
        slot.rids = []

    # -------------------------------------------------------------------- run
    def run(self, trace: dict, max_step_requests: int = 256) -> dict:
        t_arr = np.asarray(trace["t"], dtype=np.float64)
        total = t_arr.size
        nb = [request_bytes(int(n), int(b), str(d)) for n, b, d in
              zip(trace["n"], trace["batch"], trace["dtype"])]
        done_t = np.full(total, np.nan)
        pending: list[int] = []
        head = 0
        nxt = 0
        inflight = 0
        max_inflight = 0
        steps = 0
        max_busy = 0
        reqs_per_step = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        completed = 0
        while completed < total:
            now = time.perf_counter() - t0
            while nxt < total and t_arr[nxt] <= now:
                pending.append(nxt)
                nxt += 1
            progressed = False
            for s in self.slots:
                if s.busy and s.event.query():
                    tdone = time.perf_counter() - t0
                    rids = list(s.rids)
                    self._complete(s)
                    done_t[rids] = tdone
                    inflight -= sum(nb[r] for r in rids)
                    completed += len(rids)
                    progressed = True
            for s in self.slots:
                if s.busy or head >= len(pending):
                    continue
                take, head, inflight = admit_step(pending, head, trace, inflight, self.budget,
                                                  self._fits, max_step_requests, nb)
                if not take:
                    continue
                self._launch(s, take, trace)
                steps += 1
                reqs_per_step.append(len(take))
                max_inflight = max(max_inflight, inflight)
                max_busy = max(max_busy, sum(x.busy for x in self.slots))
                progressed = True
            if (head < len(pending) and not any(x.busy for x in self.slots)
                    and not progressed):
                raise RuntimeError(f"request {pending[head]} exceeds the budget or a slot's capacity")
            if head > 4096:                      # trim the admitted prefix
                pending = pending[head:]
                head = 0
            if not progressed:
                time.sleep(0)
        wall = np.nanmax(done_t) - t_arr[0]
        lat = done_t - t_arr
        out = latency_summary(lat)
        out.update({"requests": int(total), "steps": steps,
                    "mean_requests_per_step": float(np.mean(reqs_per_step)) if reqs_per_step else 0,
                    "gbs": float(np.sum(nb) / wall / 1e9), "wall_s": float(wall),
                    "max_inflight_bytes": int(max_inflight), "budget_bytes": self.budget,
                    "max_concurrent_steps": int(max_busy), "slots": len(self.slots),
                    "direct_steps": int(self.direct_steps), "direct_max": self.direct_max})
        return out


def run_per_request(trace: dict, streams: int = 4, kind: str = "dual_select", seed: int = 0,
                    budget_bytes: int = 64 << 30, keep_io: dict = None) -> dict:
    """Same trace, one launch per request (cached regular plans), round-robin
    over `streams` streams, admitted in arrival order under the same HBM
    budget as the continuous loop (request bytes in flight).

    Plans are cached per (shape, stream): a two-pass plan owns one workspace
    and must not run on two streams at once, so each stream has its own.
    ``keep_io``: a dict that receives {rid: (input, output)} device copies."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    sts = [torch.cuda.Stream() for _ in range(streams)]
    plans = {}
    t_arr = np.asarray(trace["t"], dtype=np.float64)
    total = t_arr.size
    nb = [request_bytes(int(n), int(b), str(d)) for n, b, d in
          zip(trace["n"], trace["batch"], trace["dtype"])]
    done_t = np.full(total, np.nan)
    inflight = {}
    inflight_bytes = 0
    max_inflight = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nxt, completed, k = 0, 0, 0
    while completed < total:
        now = time.perf_counter() - t0
        progressed = False
        while nxt < total and t_arr[nxt] <= now and (
                inflight_bytes + nb[nxt] <= budget_bytes or not inflight):
            n, b, dt = int(trace["n"][nxt]), int(trace["batch"][nxt]), str(trace["dtype"][nxt])
            si = k % streams
            k += 1
            st = sts[si]
            key = (n, b, dt, si)
            if key not in plans:
                plans[key] = binding.Plan(n, b, dt, kind)
            with torch.cuda.stream(st):
                buf = torch.empty((b, n, 2), dtype=TORCH_DTYPE[dt], device="cuda")
                buf.normal_(0.0, 1.0, generator=gen)
                if keep_io is not None:
                    x_in = buf.clone()
                plans[key].execute(buf, buf, stream=st)
                if keep_io is not None:
                    keep_io[nxt] = (x_in, buf)
                ev = torch.cuda.Event()
                ev.record(st)
            inflight[nxt] = (ev, buf)
            inflight_bytes += nb[nxt]
            max_inflight = max(max_inflight, inflight_bytes)
            nxt += 1
            progressed = True
        for rid in list(inflight.keys()):
            if inflight[rid][0].query():
                done_t[rid] = time.perf_counter() - t0
                del inflight[rid]
                inflight_bytes -= nb[rid]
                completed += 1
                progressed = True
        if not progressed:
            time.sleep(0)
    for p in plans.values():
        p.close()
    wall = np.nanmax(done_t) - t_arr[0]
    out = latency_summary(done_t - t_arr)
    out.update({"requests": int(total), "launches": int(total),
                "gbs": float(np.sum(nb) / wall / 1e9), "wall_s": float(wall), "streams": streams,
                "max_inflight_bytes": int(max_inflight), "budget_bytes": int(budget_bytes)})
    return out
