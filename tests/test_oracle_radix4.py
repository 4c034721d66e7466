"""Pins of the oracle's radix-4 form (Sec. VI, "Generality": every twiddle
multiplication of a radix-r butterfly takes its own min-ratio factorisation)
against what the paper and the mathematics fix (CPU only):

* the FP64 radix-4 emulation is the DFT of eq. (1) (forward and inverse,
  every size parity, several table kinds);
* every ratio the radix-4 butterflies use is at most 1 in magnitude: the
  twiddle ratios t of W^j, W^2j, W^3j (the Theorem) and the odd-pair ratio
  rho, before and after rounding, up to N = 2^20;
* worked binary16 and binary32 examples whose products are inexact
  (tests/golden/radix4_fp16_n8_inexact.txt, radix4_fp32_n8_inexact.txt) and
  one that fixes rho's rounding (tests/golden/radix4_fp16_n32_rho.txt);
* the binary16 error stays under the cumulative bound of eq. (cumulative);
* planted mistakes in the radix-4 code are caught.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 4096])
@pytest.mark.parametrize("kind", ["dual_select", "cosine", "lf_w0_exempt"])
def test_radix4_fp64_is_the_dft(n, kind):
    x = np.random.default_rng(n).standard_normal((3, n, 2))
    assert rel(oracle.emulate4(x, kind, "f64"), oracle.dft64(x)) < 1e-13
    assert rel(oracle.emulate4(x, kind, "f64", inverse=True), oracle.dft64(x, inverse=True)) < 1e-13


def test_radix4_every_ratio_at_most_one():
    for m in range(2, 21):
        n = 1 << m
        mult, ratio, path = oracle.table_count(n, 3 * n // 4, "dual_select")
        assert np.all(np.abs(ratio) <= 1.0)                       # the Theorem, k < 3N/4
        assert np.all(np.abs(mult) >= np.sqrt(0.5) * (1 - 1e-15))  # the larger of |cos|, |sin|
        rho, sel = oracle.pairs4(n, "dual_select")
        assert np.all(np.abs(rho) <= 1.0)
        for store in (np.float16, np.float32):
            assert np.all(np.abs(ratio.astype(store)) <= 1.0)
            assert np.all(np.abs(rho.astype(store)) <= 1.0)
        # the outer multiplier is the larger of the pair
        j = np.arange(n // 4)
        m1, m3 = np.abs(mult[j]), np.abs(mult[3 * j])
        assert np.array_equal(sel.astype(bool), m1 >= m3)


def test_radix4_tables_extend_the_radix2_table():
    # entries k < N/2 are Algorithm 1's table; k in [N/2, 3N/4) are W^k = -W^{k-N/2}
    # (cos and sin both flip sign: same path, same ratio, negated multiplier, up to
    # the rounding of the angle),
    # except at the 45-degree ties, where the FP64 values decide either path
    for n in (8, 64, 1024, 1 << 16):
        m4, r4, p4 = oracle.table_count(n, 3 * n // 4, "dual_select")
        m2, r2, p2 = oracle.table(n, "dual_select")
        assert np.array_equal(m4[: n // 2], m2) and np.array_equal(r4[: n // 2], r2)
        k = np.arange(n // 2, 3 * n // 4)
        tie = (8 * (k - n // 2)) % n == 0
        tie &= (k - n // 2) % (n // 4) != 0
        same = p4[k] == p2[k - n // 2]
        assert np.all(same | tie)
        assert np.allclose(m4[k][same], -m2[k - n // 2][same], rtol=0, atol=1e-14)
        assert np.allclose(r4[k][same], r2[k - n // 2][same], rtol=0, atol=1e-14)
        assert np.all(np.abs(np.abs(r4[k][~same]) - 1) < 1e-14)


def _worked(fname, dtype, npdt):
    rows = np.loadtxt(os.path.join(GOLDEN, fname))
    x = rows[:, 1:3].astype(npdt)[None]
    assert np.array_equal(x.astype(np.float64)[0], rows[:, 1:3])
    y = oracle.emulate4(x, "dual_select", dtype)[0].astype(np.float64)
    assert np.array_equal(y, rows[:, 3:5])


@pytest.mark.parametrize("fname,dtype,npdt", [("radix4_fp16_n8_inexact.txt", "f16", np.float16),
                                              ("radix4_fp32_n8_inexact.txt", "f32", np.float32)])
def test_radix4_hand_worked_n8(fname, dtype, npdt):
    _worked(fname, dtype, npdt)


def test_radix4_hand_worked_n32_rho_rounded_once():
    rows = np.loadtxt(os.path.join(GOLDEN, "radix4_fp16_n32_rho.txt"))
    x = np.zeros((1, 32, 2), np.float16)
    x[0, 1] = (-0.7744140625, 0.5234375)
    x[0, 3] = (-0.912109375, 0.275390625)
    y = oracle.emulate4(x, "dual_select", "f16")[0].astype(np.float64)
    assert np.array_equal(y[rows[:, 0].astype(int)], rows[:, 1:3])


def test_radix4_fp16_within_cumulative_bound():
    # rel-L2 against FP64 under (1 + u)^m - 1 (eq. (cumulative), |t| <= 1),
    # and of the same order as the radix-2 form's
    for n, seed in ((1024, 21), (4096, 22), (2048, 23)):
        x = np.random.default_rng(seed).uniform(-1, 1, (8, n, 2)).astype(np.float16)
        ref = oracle.fft64(x.astype(np.float64))
        e4 = oracle.errors(oracle.emulate4(x, "dual_select", "f16"), ref)
        e2 = oracle.errors(oracle.emulate(x, "dual_select", "f16"), ref)
        bound = (1 + 2.0 ** -11) ** int(np.log2(n)) - 1
        assert e4["nonfinite"] == 0 and 1e-4 < e4["rel_l2"] < bound
        assert 0.5 < e4["rel_l2"] / e2["rel_l2"] < 1.5


def test_radix4_fp32_error_level():
    n = 1024
    x = np.random.default_rng(1).standard_normal((16, n, 2)).astype(np.float32)
    ref = oracle.fft64(x.astype(np.float64))
    e = oracle.errors(oracle.emulate4(x, "dual_select", "f32"), ref)
    assert e["nonfinite"] == 0 and 3e-8 < e["rel_l2"] < 1e-6


def _radix4_pin_checks():
    def dft_check():
        for n in (64, 128):
            x = np.random.default_rng(9).standard_normal((2, n, 2))
            assert rel(oracle.emulate4(x, "dual_select", "f64"), oracle.dft64(x)) < 1e-13
    def worked16():
        _worked("radix4_fp16_n8_inexact.txt", "f16", np.float16)
    def worked32():
        _worked("radix4_fp32_n8_inexact.txt", "f32", np.float32)
    def rho_check():
        test_radix4_hand_worked_n32_rho_rounded_once()
    return [dft_check, worked16, worked32, rho_check]


@pytest.mark.parametrize("mutant", [6, 7, 8, 9])
def test_radix4_planted_mistakes_are_caught(mutant, tmp_path):
    # 6: each FMA split into a rounded product and a rounded add; 7: the sign of
    # rho in g1; 8: the sign of the j M g1 term in Y1; 9: rho left unrounded
    so = str(tmp_path / f"mut{mutant}.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    f"-DORC_MUTANT={mutant}", "-o", so, oracle._SRC, "-lm"], check=True)
    saved_lib, saved_path = oracle._lib, oracle._LIB
    try:
        oracle._lib, oracle._LIB = None, so
        caught = 0
        for check in _radix4_pin_checks():
            try:
                check()
            except AssertionError:
                caught += 1
        assert caught >= 1, f"mutant {mutant} passed every radix-4 pin"
    finally:
        oracle._lib, oracle._LIB = saved_lib, saved_path
