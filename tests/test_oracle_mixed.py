"""Pins of the oracle's binary16-storage / binary32-butterfly emulation
("f16f32") to the mathematics, not to itself: its result is the exact DFT of
the binary16 input rounded once to binary16, up to the binary32 butterflies'
error, so almost every component equals the correctly rounded DFT and none is
more than half a binary16 ulp plus that error away."""
import numpy as np
import pytest

import oracle
from paper_2604_00567_amd import inputs


def ulp16(a):
    """Spacing of binary16 values at |a| (subnormal spacing 2^-24 below 2^-14)."""
    a = np.abs(np.asarray(a, np.float64))
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -14)))
    return 2.0 ** (e - 10)


@pytest.mark.parametrize("n", [16, 256, 1024, 4096])
def test_mixed_is_the_exact_dft_rounded_once(n):
    x = inputs.uniform(n, 6, seed=n + 3, dtype="f16")
    y = oracle.emulate(x, "dual_select", "f16f32").astype(np.float64)
    exact = oracle.dft64(x.astype(np.float64)) if n <= 256 else oracle.fft64(x.astype(np.float64))
    rn = oracle.rn16(exact).astype(np.float64)
    # binary32 butterflies: error below 3 log2(n) binary32 roundings of the rms output
    m = int(np.log2(n))
    f32_err = 3 * m * 2.0 ** -24 * np.sqrt(np.mean(exact ** 2)) * np.sqrt(n)
    assert np.all(np.abs(y - exact) <= 0.5 * ulp16(exact) + f32_err)
    assert np.mean(y == rn) > 0.98         # the rest: near-ties the binary32 error crosses
    e = oracle.errors(y, exact)
    assert e["rel_l2"] < 2.0 ** -11


def test_mixed_impulse_and_constant():
    n = 1024
    x = np.zeros((2, n, 2), np.float16)
    x[0, 0, 0] = 1.0                       # impulse: all-ones spectrum, exactly
    x[1, :, 0] = 0.5                       # constant: n/2 at k = 0, zero elsewhere
    y = oracle.emulate(x, "dual_select", "f16f32")
    assert np.all(y[0, :, 0] == 1.0) and np.all(y[0, :, 1] == 0.0)
    assert y[1, 0, 0] == n / 2 and y[1, 0, 1] == 0.0
    assert np.max(np.abs(y[1, 1:].astype(np.float64))) < 1e-3


def test_mixed_is_more_accurate_than_binary16_butterflies():
    n = 1024
    x = inputs.uniform(n, 16, seed=5, dtype="f16")
    exact = oracle.fft64(x.astype(np.float64))
    e_mix = oracle.errors(oracle.emulate(x, "dual_select", "f16f32"), exact)["rel_l2"]
    e_f16 = oracle.errors(oracle.emulate(x, "dual_select", "f16"), exact)["rel_l2"]
    assert e_mix < 2.0 ** -11 < e_f16 and e_mix < 0.5 * e_f16


def test_mixed_inverse_is_the_exact_inverse_rounded_once():
    n = 512
    x = inputs.uniform(n, 4, seed=9, dtype="f16")
    y = oracle.emulate(x, "dual_select", "f16f32", inverse=True).astype(np.float64)
    exact = oracle.dft64(x.astype(np.float64), inverse=True)
    assert np.mean(y == oracle.rn16(exact).astype(np.float64)) > 0.99
