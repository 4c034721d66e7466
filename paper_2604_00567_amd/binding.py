"""ctypes binding of libdsfft.so: the C ABI of include/dsfft.h, same names.

Argument marshalling only: every FFT step runs in the HIP kernels of the
library.  Importing this module loads the library and raises if it has not
been built (there is no other path).  Torch is used only to hand device
pointers and streams through (``Plan.execute`` accepts torch tensors).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsfft.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "dsfft.h")

FFT_OK, FFT_EINVAL, FFT_ENOMEM, FFT_EHIP, FFT_EUNSUPPORTED = 0, -1, -2, -3, -4
FFT_F16, FFT_F32 = 0, 1
FFT_F16_F32 = 2           # binary16 storage, binary32 butterflies (plans only)
DTYPES = {"f16": FFT_F16, "f32": FFT_F32, "f16f32": FFT_F16_F32}
KINDS = {"dual_select": 0, "linzer_feig": 1, "cosine": 2, "lf_w0_exempt": 3}
ELEM_BYTES = {FFT_F16: 4, FFT_F32: 8, FFT_F16_F32: 4}


class FFTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dsfft error {code}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2604_00567_amd.build`")

# torch bundles its own HIP runtime under the same soname (libamdhip64.so.7).
# Loading torch first makes the library bind to that runtime, so streams and
# device pointers handed over from torch belong to the runtime the kernels are
# launched with; loading the library first would bring in a second runtime.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)
_vp, _i64, _int, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t

FFT_SERVE_CONTINUOUS, FFT_SERVE_PER_REQUEST = 0, 1


class ServeConfig(ctypes.Structure):
    """fft_serve_config."""
    _fields_ = [("mode", ctypes.c_int), ("slots", ctypes.c_int), ("kind", ctypes.c_int),
                ("direct_max", ctypes.c_int), ("max_step_requests", ctypes.c_int),
                ("max_large", ctypes.c_int), ("max_transforms", ctypes.c_int64),
                ("max_items", ctypes.c_int64), ("budget_bytes", ctypes.c_size_t),
                ("slot_bytes", ctypes.c_size_t), ("seed", ctypes.c_uint64), ("split_direct", ctypes.c_int)]


class ServeStats(ctypes.Structure):
    """fft_serve_stats."""
    _fields_ = [("steps", ctypes.c_int64), ("direct_steps", ctypes.c_int64),
                ("mean_requests_per_step", ctypes.c_double), ("max_inflight_bytes", ctypes.c_uint64),
                ("max_concurrent", ctypes.c_int), ("wall_s", ctypes.c_double)]
_SIGS = {
    "fft_last_error": ([], ctypes.c_char_p),
    "fft_plan_create": ([_i64, _i64, _int, _int], _vp),
    "fft_plan_create_variant": ([_i64, _i64, _int, _int, _int, _int, _int], _vp),
    "fft_execute": ([_vp, _vp, _vp, _vp], _int),
    "fft_execute_scratch": ([_vp, _vp, _vp, _vp], _int),
    "fft_destroy": ([_vp], None),
    "fft_table_build": ([_i64, _int, _int, _vp, _vp, _vp], _int),
    "fft_table_build_dir": ([_i64, _int, _int, _int, _vp, _vp, _vp], _int),
    "fft_plan_create_dir": ([_i64, _i64, _int, _int, _int], _vp),
    "fft_plan_create_radix4": ([_i64, _i64, _int, _int, _int, _int], _vp),
    "fft_config_count_radix4": ([_i64, _int, ctypes.POINTER(_int)], _int),
    "fft_table_build_radix4": ([_i64, _int, _int, _int, _vp, _vp, _vp, _vp, _vp], _int),
    "fft_plan_info": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_int),
                       ctypes.POINTER(_int), ctypes.c_char_p, _sz], _int),
    "fft_plan_workspace_bytes": ([_vp, ctypes.POINTER(_sz)], _int),
    "fft_plan_set_workspace": ([_vp, _vp, _sz], _int),
    "fft_config_count": ([_i64, _int, ctypes.POINTER(_int), ctypes.POINTER(_int),
                          ctypes.POINTER(_int)], _int),
    "fft_batch_create": ([_vp, _i64, _int, _int], _vp),
    "fft_batch_create_tuned": ([_vp, _i64, _int, _int, _int, _int], _vp),
    "fft_batch_create_classes": ([_vp, _i64, _int, _int, _vp], _vp),
    "fft_batch_tune_classes": ([_int, _int, _int, _vp], _int),
    "fft_batch_execute": ([_vp, _vp, _vp, _vp], _int),
    "fft_batch_elements": ([_vp, ctypes.POINTER(_i64)], _int),
    "fft_batch_info": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_sz)], _int),
    "fft_batch_destroy": ([_vp], None),
    "fft_batch_work_list": ([_vp, _i64, _int, _vp, _i64, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                             _vp, _i64, ctypes.POINTER(_i64), _vp, _i64, ctypes.POINTER(_i64),
                             ctypes.POINTER(_i64)], _int),
    "fft_tune": ([_i64, _i64, _int, _int, _int, ctypes.c_char_p, _sz], _int),
    "fft_tuned_choice": ([_i64, _int, ctypes.POINTER(_int), ctypes.POINTER(_int),
                          ctypes.POINTER(_int)], _int),
    "fft_batch_tune": ([_int, _int, _int, ctypes.POINTER(_int), ctypes.POINTER(_int)], _int),
    "fft_serve_slot_create": ([_int, _int, _i64, _i64, _int, _sz], _vp),
    "fft_serve_slot_launch": ([_vp, _vp, _vp, _vp, _i64, _vp, _vp], _int),
    "fft_serve_slot_query": ([_vp], _int),
    "fft_serve_slot_destroy": ([_vp], None),
    "fft_serve_run": ([ctypes.POINTER(ServeConfig), _vp, _vp, _vp, _vp, _i64, _vp, ctypes.POINTER(ServeStats),
                       _vp, _vp], _int),
    "fft_serve_fill": ([_int, _vp, _i64, ctypes.c_uint64, ctypes.c_uint64, _vp], _int),
    "fft_serve_admit": ([_vp, _vp, _vp, _i64, _i64, _sz, ctypes.POINTER(ServeConfig), _vp,
                         ctypes.POINTER(_i64), ctypes.POINTER(_sz)], _int),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def declared_functions() -> list[str]:
    """Function names declared in include/dsfft.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fft_[a-z_0-9]+)\s*\(", text)))


def _dt(dtype) -> int:
    return DTYPES[dtype] if isinstance(dtype, str) else int(dtype)


def _kd(kind) -> int:
    return KINDS[kind] if isinstance(kind, str) else int(kind)


def fft_last_error() -> str:
    return _lib.fft_last_error().decode()


def _check(rc: int):
    if rc != FFT_OK:
        raise FFTError(rc, fft_last_error())


def fft_plan_create(n: int, batch: int, dtype, kind) -> int:
    h = _lib.fft_plan_create(n, batch, _dt(dtype), _kd(kind))
    if not h:
        raise FFTError(FFT_EINVAL, fft_last_error())
    return h


FFT_FORWARD, FFT_INVERSE = -1, 1
_DIRECTIONS = {"forward": FFT_FORWARD, "inverse": FFT_INVERSE}


def _dir(direction) -> int:
    return _DIRECTIONS[direction] if isinstance(direction, str) else int(direction)


def fft_plan_create_dir(n: int, batch: int, dtype, kind, direction) -> int:
    h = _lib.fft_plan_create_dir(n, batch, _dt(dtype), _kd(kind), _dir(direction))
    if not h:
        raise FFTError(FFT_EINVAL, fft_last_error())
    return h


def fft_plan_create_variant(n: int, batch: int, dtype, kind, variant_a: int = 0,
                            variant_b: int = 0, two_pass: bool = False) -> int:
    h = _lib.fft_plan_create_variant(n, batch, _dt(dtype), _kd(kind), variant_a, variant_b,
                                     1 if two_pass else 0)
    if not h:
        raise FFTError(FFT_EUNSUPPORTED, fft_last_error())
    return h


def fft_execute(plan: int, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    _check(_lib.fft_execute(plan, in_ptr, out_ptr, stream))


def fft_execute_scratch(plan: int, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    _check(_lib.fft_execute_scratch(plan, in_ptr, out_ptr, stream))


def fft_destroy(plan: int) -> None:
    _lib.fft_destroy(plan)


def fft_table_build(n: int, dtype, kind, direction="forward"):
    """(mult, ratio, path) of the size-n table rounded to dtype (host only)."""
    dt = _dt(dtype)
    h = n // 2
    st = np.uint16 if dt == FFT_F16 else np.float32
    mult = np.empty(h, st)
    ratio = np.empty(h, st)
    path = np.empty(h, np.uint8)
    _check(_lib.fft_table_build_dir(n, dt, _kd(kind), _dir(direction), mult.ctypes.data,
                                    ratio.ctypes.data, path.ctypes.data))
    if dt == FFT_F16:
        mult, ratio = mult.view(np.float16), ratio.view(np.float16)
    return mult, ratio, path


def fft_table_build_radix4(n: int, dtype, kind, direction="forward"):
    """Radix-4 export (host only): (mult, ratio, path) of W^k for k < 3n/4 and
    (rho, sel) per column j < n/4 of the last stage, rounded to dtype."""
    dt = _dt(dtype)
    st = np.uint16 if dt == FFT_F16 else np.float32
    k3, k1 = 3 * n // 4, n // 4
    mult, ratio, path = np.empty(k3, st), np.empty(k3, st), np.empty(k3, np.uint8)
    rho, sel = np.empty(k1, st), np.empty(k1, np.uint8)
    _check(_lib.fft_table_build_radix4(n, dt, _kd(kind), _dir(direction), mult.ctypes.data,
                                       ratio.ctypes.data, path.ctypes.data, rho.ctypes.data,
                                       sel.ctypes.data))
    if dt == FFT_F16:
        mult, ratio, rho = mult.view(np.float16), ratio.view(np.float16), rho.view(np.float16)
    return mult, ratio, path, rho, sel


def fft_plan_create_radix4(n: int, batch: int, dtype, kind, direction="forward",
                           variant: int = -1) -> int:
    h = _lib.fft_plan_create_radix4(n, batch, _dt(dtype), _kd(kind), _dir(direction), variant)
    if not h:
        raise FFTError(FFT_EUNSUPPORTED, fft_last_error())
    return h


def fft_config_count_radix4(n: int, dtype) -> int:
    c = _int()
    _check(_lib.fft_config_count_radix4(n, _dt(dtype), ctypes.byref(c)))
    return c.value


def fft_plan_info(plan: int) -> dict:
    n, b = _i64(), _i64()
    d, k = _int(), _int()
    buf = ctypes.create_string_buffer(512)
    _check(_lib.fft_plan_info(plan, ctypes.byref(n), ctypes.byref(b), ctypes.byref(d),
                              ctypes.byref(k), buf, 512))
    return {"n": n.value, "batch": b.value, "dtype": d.value, "kind": k.value,
            "config": buf.value.decode()}


def fft_plan_workspace_bytes(plan: int) -> int:
    s = _sz()
    _check(_lib.fft_plan_workspace_bytes(plan, ctypes.byref(s)))
    return s.value


def fft_plan_set_workspace(plan: int, dev_ptr: int, nbytes: int) -> None:
    _check(_lib.fft_plan_set_workspace(plan, dev_ptr, nbytes))


def fft_config_count(n: int, dtype) -> tuple[int, int, int]:
    a, b, c = _int(), _int(), _int()
    _check(_lib.fft_config_count(n, _dt(dtype), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def fft_tune(n: int, batch: int, dtype, kind="dual_select", reps: int = 10) -> list:
    """Times every configuration for (n, dtype); returns the candidates' report."""
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    _check(_lib.fft_tune(n, batch, _dt(dtype), _kd(kind), reps, buf, 1 << 16))
    return json.loads(buf.value.decode())


def fft_tuned_choice(n: int, dtype):
    a, b, t = _int(), _int(), _int()
    rc = _lib.fft_tuned_choice(n, _dt(dtype), ctypes.byref(a), ctypes.byref(b), ctypes.byref(t))
    if rc != FFT_OK:
        return None
    return a.value, b.value, bool(t.value)


def fft_batch_tune(dtype, kind="dual_select", reps: int = 5) -> tuple[int, int]:
    a, b = _int(), _int()
    _check(_lib.fft_batch_tune(_dt(dtype), _kd(kind), reps, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def fft_batch_tune_classes(dtype, kind="dual_select", reps: int = 5) -> list[int]:
    """Per log2 N (0..14): 1 where the batch tuner picked the alternative configuration."""
    alt = np.zeros(15, np.int32)
    _check(_lib.fft_batch_tune_classes(_dt(dtype), _kd(kind), reps, alt.ctypes.data))
    return alt.tolist()


def fft_batch_create(sizes, dtype, kind, choice=None) -> int:
    """choice: None (defaults), (choice_1024, choice_4096), or 15 per-class flags."""
    arr = np.ascontiguousarray(np.asarray(sizes, dtype=np.int64))
    if choice is None:
        h = _lib.fft_batch_create(arr.ctypes.data, arr.size, _dt(dtype), _kd(kind))
    elif len(choice) == 15:
        alt = np.ascontiguousarray(np.asarray(choice, dtype=np.int32))
        h = _lib.fft_batch_create_classes(arr.ctypes.data, arr.size, _dt(dtype), _kd(kind), alt.ctypes.data)
    else:
        h = _lib.fft_batch_create_tuned(arr.ctypes.data, arr.size, _dt(dtype), _kd(kind),
                                        int(choice[0]), int(choice[1]))
    if not h:
        raise FFTError(FFT_EINVAL, fft_last_error())
    return h


def fft_batch_execute(batch: int, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    _check(_lib.fft_batch_execute(batch, in_ptr, out_ptr, stream))


def fft_batch_elements(batch: int) -> int:
    v = _i64()
    _check(_lib.fft_batch_elements(batch, ctypes.byref(v)))
    return v.value


def fft_batch_info(batch: int) -> dict:
    it, gr, ws = _i64(), _i64(), _sz()
    _check(_lib.fft_batch_info(batch, ctypes.byref(it), ctypes.byref(gr), ctypes.byref(ws)))
    return {"items": it.value, "grid": gr.value, "workspace_bytes": ws.value}


def fft_batch_destroy(batch: int) -> None:
    _lib.fft_batch_destroy(batch)


WORK_FIELDS = ("cfg", "nunits", "first", "log_m", "phase", "slot", "in_off", "out_off")


def fft_batch_work_list(sizes, dtype="f16"):
    """The work list of an uneven batch (host only): (items (k, 8) int64 with
    columns WORK_FIELDS, number of phase-0 items, whole-transform offsets,
    list-kernel offsets, workspace elements)."""
    arr = np.ascontiguousarray(np.asarray(sizes, dtype=np.int64))
    ni, p0, no, nl, ws = _i64(), _i64(), _i64(), _i64(), _i64()
    dt = _dt(dtype)
    _check(_lib.fft_batch_work_list(arr.ctypes.data, arr.size, dt, None, 0, ctypes.byref(ni),
                                    ctypes.byref(p0), None, 0, ctypes.byref(no), None, 0,
                                    ctypes.byref(nl), ctypes.byref(ws)))
    items = np.zeros((ni.value, 8), np.int64)
    offs = np.zeros(max(1, no.value), np.int64)
    lst = np.zeros(max(1, nl.value), np.int64)
    _check(_lib.fft_batch_work_list(arr.ctypes.data, arr.size, dt, items.ctypes.data, ni.value,
                                    ctypes.byref(ni), ctypes.byref(p0), offs.ctypes.data, offs.size,
                                    ctypes.byref(no), lst.ctypes.data, lst.size, ctypes.byref(nl),
                                    ctypes.byref(ws)))
    return items, p0.value, offs[:no.value], lst[:nl.value], ws.value


def fft_serve_slot_create(dtype, kind, max_items: int, max_transforms: int, max_large: int,
                          ws_bytes: int) -> int:
    h = _lib.fft_serve_slot_create(_dt(dtype), _kd(kind), max_items, max_transforms, max_large,
                                   ws_bytes)
    if not h:
        raise FFTError(FFT_ENOMEM, fft_last_error())
    return h


def fft_serve_slot_launch(slot: int, n, batch, off, data_ptr: int, stream: int = 0) -> None:
    n = np.ascontiguousarray(n, dtype=np.int64)
    batch = np.ascontiguousarray(batch, dtype=np.int64)
    off = np.ascontiguousarray(off, dtype=np.int64)
    assert n.size == batch.size == off.size
    _check(_lib.fft_serve_slot_launch(slot, n.ctypes.data, batch.ctypes.data, off.ctypes.data,
                                      n.size, data_ptr, stream))


def fft_serve_slot_query(slot: int) -> bool:
    rc = _lib.fft_serve_slot_query(slot)
    if rc < 0:
        raise FFTError(rc, fft_last_error())
    return rc == 1


def fft_serve_slot_destroy(slot: int) -> None:
    _lib.fft_serve_slot_destroy(slot)


# ----------------------------------------------------------- torch marshalling

def _torch_stream(stream) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check_tensor(t, n: int, batch: int, dt: int):
    import torch
    f16_stored = dt in (FFT_F16, FFT_F16_F32)
    want = torch.float16 if f16_stored else torch.float32
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    ok_dtype = t.dtype == want or (dt == FFT_F32 and t.dtype == torch.complex64) or \
        (f16_stored and t.dtype == torch.complex32)
    if not ok_dtype:
        raise ValueError(f"tensor dtype {t.dtype} does not match the plan")
    if t.numel() * t.element_size() != n * batch * ELEM_BYTES[dt]:
        raise ValueError("tensor size does not match n * batch complex elements")


class Plan:
    """Owns a plan handle; execute() takes torch tensors laid out (batch, n, 2)."""

    def __init__(self, n: int, batch: int, dtype="f16", kind="dual_select", variant=None,
                 direction="forward", radix: int = 2):
        self.n, self.batch, self.dtype, self.kind = n, batch, _dt(dtype), _kd(kind)
        self.direction = _dir(direction)
        if radix == 4:
            self.handle = fft_plan_create_radix4(n, batch, self.dtype, self.kind, self.direction,
                                                 -1 if variant is None else int(variant))
        elif radix != 2:
            raise FFTError(FFT_EINVAL, "radix must be 2 or 4")
        elif variant is None:
            self.handle = fft_plan_create_dir(n, batch, self.dtype, self.kind, self.direction)
        elif self.direction == FFT_FORWARD:
            self.handle = fft_plan_create_variant(n, batch, self.dtype, self.kind, *variant)
        else:
            raise FFTError(FFT_EINVAL, "explicit kernel variants are forward-only")

    def execute(self, x, y, stream=None) -> None:
        _check_tensor(x, self.n, self.batch, self.dtype)
        _check_tensor(y, self.n, self.batch, self.dtype)
        fft_execute(self.handle, x.data_ptr(), y.data_ptr(), _torch_stream(stream))

    def execute_scratch(self, x, y, stream=None) -> None:
        """fft_execute_scratch: the same transform with no device allocation."""
        _check_tensor(x, self.n, self.batch, self.dtype)
        _check_tensor(y, self.n, self.batch, self.dtype)
        fft_execute_scratch(self.handle, x.data_ptr(), y.data_ptr(), _torch_stream(stream))

    def info(self) -> dict:
        return fft_plan_info(self.handle)

    def close(self) -> None:
        if self.handle:
            fft_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Owns an uneven-size batch; execute() takes packed torch tensors (total, 2)."""

    def __init__(self, sizes, dtype="f16", kind="dual_select", choice=None):
        self.sizes = np.asarray(sizes, dtype=np.int64)
        self.dtype, self.kind = _dt(dtype), _kd(kind)
        self.handle = fft_batch_create(self.sizes, self.dtype, self.kind, choice)
        self.total = fft_batch_elements(self.handle)

    def execute(self, x, y, stream=None) -> None:
        _check_tensor(x, self.total, 1, self.dtype)
        _check_tensor(y, self.total, 1, self.dtype)
        fft_batch_execute(self.handle, x.data_ptr(), y.data_ptr(), _torch_stream(stream))

    def info(self) -> dict:
        return fft_batch_info(self.handle)

    def close(self) -> None:
        if self.handle:
            fft_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _trace_arrays(trace):
    t = np.ascontiguousarray(trace["t"], dtype=np.float64)
    n = np.ascontiguousarray(trace["n"], dtype=np.int64)
    b = np.ascontiguousarray(trace["batch"], dtype=np.int64)
    d = np.ascontiguousarray([_dt(str(x)) for x in trace["dtype"]], dtype=np.int32)
    return t, n, b, d


def fft_serve_run(cfg: ServeConfig, trace, out_dev: int = 0, out_off=None):
    """Runs the native serving loop over `trace` (dict of t, n, batch, dtype);
    returns (done_t seconds per request, ServeStats)."""
    t, n, b, d = _trace_arrays(trace)
    done = np.empty(t.size, np.float64)
    st = ServeStats()
    off = None if out_off is None else np.ascontiguousarray(out_off, dtype=np.int64)
    _check(_lib.fft_serve_run(ctypes.byref(cfg), t.ctypes.data, n.ctypes.data, b.ctypes.data, d.ctypes.data,
                              t.size, done.ctypes.data, ctypes.byref(st), out_dev or None,
                              None if off is None else off.ctypes.data))
    return done, st


def fft_serve_fill(dtype, data_ptr: int, elems: int, first: int, seed: int, stream: int = 0) -> None:
    _check(_lib.fft_serve_fill(_dt(dtype), data_ptr, elems, first, seed, stream))


def fft_serve_admit(trace, head: int, inflight_bytes: int, cfg: ServeConfig):
    """Host-only admission of one continuous step: (taken indices, bytes in flight)."""
    _, n, b, d = _trace_arrays(dict(trace, t=np.zeros(len(trace["n"]))))
    taken = np.empty(max(1, cfg.max_step_requests), np.int64)
    nt, infl = _i64(), _sz()
    _check(_lib.fft_serve_admit(n.ctypes.data, b.ctypes.data, d.ctypes.data, n.size, head, inflight_bytes,
                                ctypes.byref(cfg), taken.ctypes.data, ctypes.byref(nt), ctypes.byref(infl)))
    return taken[:nt.value].tolist(), infl.value
