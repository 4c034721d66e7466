"""Seeded synthetic inputs for the batched FFT workloads.

This module holds no FFT arithmetic: it only draws random numbers (numpy PCG64,
``default_rng(seed)``) and rounds them once, round-to-nearest-even, from FP64 to
the storage precision.  Both the tests/oracle side and the GPU side take their
inputs from here; it imports nothing else from the package.

Layout of every array: interleaved complex, shape ``(batch, n, 2)``.

Workload recipes (the paper names no dataset; its radar and neural-network
applications are stood in for by these synthetic shapes):

* ``normal``: re, im i.i.d. N(0, 1)                 (FP32 single-size case, serving)
* ``uniform``: re, im i.i.d. uniform[-1, 1)          (batched FP16 fixed-size, uneven batch)
* ``tones``: sum of 8 unit tones exp(+j 2 pi f n / N) with distinct integer
  f uniform in [0, N), plus complex N(0, 0.01^2) noise per component (large-N sweep);
  for FP16 an exact power-of-two prescale 2^-max(0, log2 N - 12) keeps the
  unnormalised transform inside the binary16 range.
* ``uneven_sizes``: N = 2^U with U uniform over an integer range (log-uniform N).
"""
from __future__ import annotations

import numpy as np

_DT = {"f16": np.float16, "f32": np.float32, "f64": np.float64}


def storage_dtype(dtype: str):
    return _DT[dtype]


def _round(x64: np.ndarray, dtype: str) -> np.ndarray:
    # numpy's float64 -> float16 / float32 casts are single round-to-nearest-even
    return np.ascontiguousarray(x64.astype(_DT[dtype]))


def normal(n: int, batch: int, seed: int, dtype: str = "f32") -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _round(rng.standard_normal((batch, n, 2)), dtype)


def uniform(n: int, batch: int, seed: int, dtype: str = "f16") -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _round(rng.uniform(-1.0, 1.0, (batch, n, 2)), dtype)


def tone_prescale(n: int, dtype: str) -> float:
    if dtype != "f16":
        return 1.0
    m = int(np.log2(n))
    return float(2.0 ** -max(0, m - 12))


def tones(n: int, batch: int, seed: int, dtype: str = "f16", ntones: int = 8,
          noise_sigma: float = 0.01) -> np.ndarray:
    rng = np.random.default_rng(seed)
    k = min(ntones, n)
    # k distinct integer frequencies per transform (rows with a repeat are redrawn)
    f = rng.integers(0, n, (batch, k))
    while True:
        srt = np.sort(f, axis=1)
        bad = np.flatnonzero(np.any(srt[:, 1:] == srt[:, :-1], axis=1)) if k > 1 else []
        if len(bad) == 0:
            break
        f[bad] = rng.integers(0, n, (len(bad), k))
    out = np.empty((batch, n, 2), np.float64)
    rows = max(1, (1 << 22) // n)
    for b0 in range(0, batch, rows):
        fb = f[b0:b0 + rows]
        # sum_f exp(+j 2 pi f t / N), synthesised as N * ifft of unit spikes at f
        spec = np.zeros((fb.shape[0], n), np.complex128)
        np.put_along_axis(spec, fb, 1.0, axis=1)
        sig = np.fft.ifft(spec, axis=1) * n
        out[b0:b0 + rows, :, 0] = sig.real
        out[b0:b0 + rows, :, 1] = sig.imag
    out += rng.normal(0.0, noise_sigma, out.shape)
    out *= tone_prescale(n, dtype)
    return _round(out, dtype)


def uneven_sizes(count: int, seed: int, log_lo: int = 6, log_hi: int = 16) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (np.int64(1) << rng.integers(log_lo, log_hi + 1, size=count)).astype(np.int64)


def packed_uniform(sizes, seed: int, dtype: str = "f16") -> np.ndarray:
    """Concatenated interleaved-complex payload for an uneven batch: shape (sum(N), 2)."""
    rng = np.random.default_rng(seed)
    total = int(np.sum(sizes))
    return _round(rng.uniform(-1.0, 1.0, (total, 2)), dtype)


def poisson_trace(rate_per_s: float, duration_s: float, seed: int, log_lo: int = 8,
                  log_hi: int = 18, batch_lo: int = 1, batch_hi: int = 64,
                  frac_f16: float = 0.75):
    """Arrival times and request shapes for the serving workload."""
    rng = np.random.default_rng(seed)
    t, times = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            break
        times.append(t)
    k = len(times)
    logn = rng.integers(log_lo, log_hi + 1, size=k)
    batch = rng.integers(batch_lo, batch_hi + 1, size=k)
    f16 = rng.random(k) < frac_f16
    return {
        "t": np.asarray(times, np.float64),
        "n": (np.int64(1) << logn).astype(np.int64),
        "batch": batch.astype(np.int64),
        "dtype": np.where(f16, "f16", "f32"),
    }
