"""Oracle for the dual-select FMA-butterfly FFT (arXiv 2604.00567).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP library
and its Python binding never import it, and the two share no code.

It wraps ``oracle_core.c`` (plain C, FP64, OpenMP over the batch), built with
gcc into ``oracle/_liboracle.so``:

* ``table(n, kind, inverse)``: FP64 twiddle table -- Algorithm 1 (dual-select),
  the epsilon-clamped Linzer-Feig table of Sec. II-B, the cosine table of
  Sec. II-C, and Linzer-Feig with W^0 exempted; ``inverse=True`` applies the
  same rules to the conjugate twiddles W^{-k} (the inverse transform);
* ``dft64`` (eq. (1) written out), ``fft64`` (radix-2 Stockham, 10-flop butterfly
  of eqs. (std1)-(std2));
* ``emulate_f16`` / ``emulate_f32`` / ``emulate_f64``: the radix-2 Stockham pass
  order with every butterfly as the six FMAs of eqs. (berg-s)-(berg-B) or
  (lf-s)-(lf-B), each FMA rounded once to the working precision (and
  ``emulate(..., "f16f32")``: binary16 data, binary32 butterflies, one rounding
  of each result to binary16);
* ``emulate4``: the radix-4 form (Sec. VI generality): canonical radix-4
  Stockham order, 22-FMA butterflies whose twiddle multiplications each take
  their own min-ratio entry, every FMA rounded once;
* ``errors``: relative L2, max-abs (complex modulus) and non-finite count;
* ``analytic_bounds``: per-butterfly and cumulative bounds of eqs.
  (per-butterfly-error) and (cumulative), as printed in Tables I-II.

Arrays use interleaved complex layout ``(batch, n, 2)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_core.c")
_LIB = os.path.join(_HERE, "_liboracle.so")

KINDS = {"dual_select": 0, "linzer_feig": 1, "cosine": 2, "lf_w0_exempt": 3}
PATH_COS, PATH_SIN = 0, 1
EPS_CLAMP = 1e-7

_lib = None


def build(force: bool = False) -> str:
    """Compile oracle_core.c with gcc (FP-contraction off, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i64, i32, dp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    for name, args in {
        "orc_table_dir": [i64, i32, i32, dp, dp, dp],
        "orc_fft64": [i64, i64, i32, dp, dp],
        "orc_dft64": [i64, i64, i32, dp, dp],
        "orc_emulate_f64": [i64, i64, i32, i32, dp, dp],
        "orc_emulate_f32": [i64, i64, i32, i32, dp, dp],
        "orc_emulate_f16": [i64, i64, i32, i32, dp, dp],
        "orc_emulate4_f64": [i64, i64, i32, i32, dp, dp],
        "orc_emulate4_f32": [i64, i64, i32, i32, dp, dp],
        "orc_emulate4_f16": [i64, i64, i32, i32, dp, dp],
        "orc_table_count": [i64, i32, i32, i64, dp, dp, dp],
        "orc_pairs4": [i64, i32, i32, dp, dp],
        "orc_rn16_array": [i64, dp, dp],
        "orc_f16_to_double_array": [i64, dp, dp],
    }.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int if name.startswith(("orc_table", "orc_fft", "orc_dft", "orc_emu",
                                                     "orc_pairs")) else None
    lib.orc_fma16.argtypes = [ctypes.c_double] * 3
    lib.orc_fma16.restype = ctypes.c_double
    lib.orc_fma32.argtypes = [ctypes.c_float] * 3
    lib.orc_fma32.restype = ctypes.c_float
    lib.orc_theta.argtypes = [i64, i64]
    lib.orc_theta.restype = ctypes.c_double
    lib.orc_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _kind(kind) -> int:
    return KINDS[kind] if isinstance(kind, str) else int(kind)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def theta(k: int, n: int) -> float:
    return float(_load().orc_theta(k, n))


def table(n: int, kind="dual_select", inverse: bool = False):
    """FP64 table for k in [0, n/2): (mult, ratio, path) with path 0 = cos, 1 = sin.
    ``inverse``: the table of the inverse transform (conjugate twiddles)."""
    lib = _load()
    h = n // 2
    mult = np.empty(h, np.float64)
    ratio = np.empty(h, np.float64)
    path = np.empty(h, np.int32)
    if lib.orc_table_dir(n, _kind(kind), int(inverse), _ptr(mult), _ptr(ratio), _ptr(path)) != 0:
        raise ValueError(f"bad table request n={n} kind={kind}")
    return mult, ratio, path


def _as_batch(x: np.ndarray, dtype) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=dtype)
    if x.ndim == 2:
        x = x[None]
    assert x.ndim == 3 and x.shape[2] == 2, "expected (batch, n, 2)"
    return x


def fft64(x: np.ndarray, inverse: bool = False) -> np.ndarray:
    """Radix-2 Stockham FFT in FP64 with the standard 10-flop butterfly
    (``inverse``: twiddles W^{-k}, unnormalised)."""
    x = _as_batch(x, np.float64)
    out = np.empty_like(x)
    if _load().orc_fft64(x.shape[1], x.shape[0], int(inverse), _ptr(x), _ptr(out)) != 0:
        raise ValueError("fft64 failed")
    return out


def dft64(x: np.ndarray, inverse: bool = False) -> np.ndarray:
    """Brute-force O(N^2) DFT of eq. (1) in FP64 (``inverse``: exponent sign +)."""
    x = _as_batch(x, np.float64)
    out = np.empty_like(x)
    if _load().orc_dft64(x.shape[1], x.shape[0], int(inverse), _ptr(x), _ptr(out)) != 0:
        raise ValueError("dft64 failed")
    return out


def emulate(x: np.ndarray, kind="dual_select", prec: str = "f16", inverse: bool = False) -> np.ndarray:
    """Six-FMA butterfly FFT with every FMA rounded once to ``prec``
    (``inverse``: the inverse transform, with the conjugate tables).

    ``x`` holds values of the working precision: float16 for "f16", float32 for
    "f32", float64 for "f64"; the result has the same dtype.

    "f16f32" (binary16 storage, binary32 butterflies): ``x`` holds float16
    values; they are widened exactly to binary32, transformed with every FMA
    rounded once to binary32 and the binary32 table, and each result is
    rounded once to binary16 (round to nearest even).
    """
    lib = _load()
    inv = int(inverse)
    if prec == "f16f32":
        x16 = _as_batch(x, np.float16)
        y32 = emulate(x16.astype(np.float32), kind, "f32", inverse)
        return rn16(y32.astype(np.float64)).reshape(y32.shape)
    if prec == "f16":
        x = _as_batch(x, np.float16)
        out = np.empty_like(x)
        rc = lib.orc_emulate_f16(x.shape[1], x.shape[0], _kind(kind), inv, _ptr(x), _ptr(out))
    elif prec == "f32":
        x = _as_batch(x, np.float32)
        out = np.empty_like(x)
        rc = lib.orc_emulate_f32(x.shape[1], x.shape[0], _kind(kind), inv, _ptr(x), _ptr(out))
    elif prec == "f64":
        x = _as_batch(x, np.float64)
        out = np.empty_like(x)
        rc = lib.orc_emulate_f64(x.shape[1], x.shape[0], _kind(kind), inv, _ptr(x), _ptr(out))
    else:
        raise ValueError(prec)
    if rc != 0:
        raise ValueError("emulation failed")
    return out


def emulate4(x: np.ndarray, kind="dual_select", prec: str = "f16", inverse: bool = False) -> np.ndarray:
    """Radix-4 form of the method (Sec. VI, generality): the canonical radix-4
    Stockham order (a radix-2 stage of span 2 first when log2 N is odd), each
    radix-4 butterfly as 22 FMAs whose three twiddle multiplications take
    their own table entries and whose odd pair takes the larger multiplier
    with the ratio |rho| <= 1; every FMA rounded once to ``prec``."""
    lib = _load()
    inv = int(inverse)
    if prec == "f16":
        x = _as_batch(x, np.float16)
        out = np.empty_like(x)
        rc = lib.orc_emulate4_f16(x.shape[1], x.shape[0], _kind(kind), inv, _ptr(x), _ptr(out))
    elif prec == "f32":
        x = _as_batch(x, np.float32)
        out = np.empty_like(x)
        rc = lib.orc_emulate4_f32(x.shape[1], x.shape[0], _kind(kind), inv, _ptr(x), _ptr(out))
    elif prec == "f64":
        x = _as_batch(x, np.float64)
        out = np.empty_like(x)
        rc = lib.orc_emulate4_f64(x.shape[1], x.shape[0], _kind(kind), inv, _ptr(x), _ptr(out))
    else:
        raise ValueError(prec)
    if rc != 0:
        raise ValueError("radix-4 emulation failed")
    return out


def table_count(n: int, count: int, kind="dual_select", inverse: bool = False):
    """FP64 table entries of W^k for k < count (the radix-4 form uses
    count = 3n/4): (mult, ratio, path)."""
    lib = _load()
    mult = np.empty(count, np.float64)
    ratio = np.empty(count, np.float64)
    path = np.empty(count, np.int32)
    if lib.orc_table_count(n, _kind(kind), int(inverse), count, _ptr(mult), _ptr(ratio), _ptr(path)) != 0:
        raise ValueError(f"bad table request n={n} count={count}")
    return mult, ratio, path


def pairs4(n: int, kind="dual_select", inverse: bool = False):
    """Odd-pair choice of the radix-4 butterflies of span n, j < n/4:
    (rho, sel) with sel = 1 where W^j's multiplier is the outer one."""
    lib = _load()
    rho = np.empty(n // 4, np.float64)
    sel = np.empty(n // 4, np.int32)
    if lib.orc_pairs4(n, _kind(kind), int(inverse), _ptr(rho), _ptr(sel)) != 0:
        raise ValueError(f"bad pair request n={n}")
    return rho, sel


def rn16(x: np.ndarray) -> np.ndarray:
    """Direct double -> binary16 round-to-nearest-even (hand-written bit routine)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(x.shape, np.float16)
    _load().orc_rn16_array(x.size, _ptr(x), _ptr(out))
    return out


def fma16(a: float, b: float, c: float) -> float:
    return float(_load().orc_fma16(a, b, c))


def fma32(a: float, b: float, c: float) -> float:
    return float(_load().orc_fma32(a, b, c))


def rounded_table(n: int, kind="dual_select", prec: str = "f16", inverse: bool = False):
    """The table rounded once from FP64 to the working precision."""
    mult, ratio, path = table(n, kind, inverse)
    if prec == "f16":
        return rn16(mult), rn16(ratio), path
    if prec == "f32":
        return mult.astype(np.float32), ratio.astype(np.float32), path
    return mult, ratio, path


def errors(y: np.ndarray, ref: np.ndarray) -> dict:
    """Relative L2 and max-abs error (complex modulus) of y against ref, plus the
    number of complex outputs with a non-finite component."""
    y = np.asarray(y, np.float64).reshape(-1, 2)
    ref = np.asarray(ref, np.float64).reshape(-1, 2)
    nonfinite = int(np.count_nonzero(~np.isfinite(y).all(axis=1)))
    d = y - ref
    dm = np.hypot(d[:, 0], d[:, 1])
    with np.errstate(invalid="ignore", over="ignore"):
        num = float(np.sqrt(np.sum(dm * dm)))
        den = float(np.sqrt(np.sum(ref * ref)))
        rel = num / den if den > 0 else (0.0 if num == 0 else float("inf"))
    return {"rel_l2": rel if nonfinite == 0 else float("nan"),
            "max_abs": float(np.max(dm)) if (dm.size and nonfinite == 0) else (float("nan") if nonfinite else 0.0),
            "nonfinite": nonfinite,
            "count": int(y.shape[0])}


UNIT_ROUNDOFF = {"f16": 2.0 ** -11, "f32": 2.0 ** -24}


def max_ratio(n: int, kind="dual_select", exclude_clamped: bool = True):
    """Largest |ratio| over the table and where it occurs.  For the clamped
    Linzer-Feig table the k=0 entry is the singularity Table I counts apart,
    so it is excluded by default."""
    mult, ratio, path = table(n, kind)
    r = np.abs(ratio)
    if exclude_clamped and _kind(kind) == KINDS["linzer_feig"]:
        r = r.copy()
        r[0] = 0.0
    k = int(np.argmax(r))
    return float(r[k]), k


def analytic_bounds(n: int, tmax: float, prec: str = "f16"):
    """Per-butterfly |t|max * u and cumulative (1 + |t|max u)^m - 1 (Sec. IV)."""
    u = UNIT_ROUNDOFF[prec]
    m = int(np.log2(n))
    return tmax * u, (1.0 + tmax * u) ** m - 1.0
