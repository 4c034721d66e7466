"""Pins of the oracle against what the paper and mathematics fix (CPU only).

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden/paper_facts.txt), a hand-worked FP16 example
(tests/golden/fp16_n4_worked.txt) and two N = 8 examples whose products are
inexact (tests/golden/fp16_n8_inexact.txt, fp32_n8_inexact.txt), closed forms, Parseval, linearity, the DFT
written out, numpy's FFT, numpy's binary16 cast and exact rational rounding.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests.exact import HALF, SINGLE, rne

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _facts():
    out = {}
    with open(os.path.join(GOLDEN, "paper_facts.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()[:2]
                out[k] = float(v)
    return out


FACTS = _facts()


def cplx(y):
    y = np.asarray(y, np.float64)
    return y[..., 0] + 1j * y[..., 1]


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


# ------------------------------------------------------------- binary16 rounding

def test_rn16_matches_numpy_cast():
    rng = np.random.default_rng(11)
    parts = [
        rng.standard_normal(20000) * 10.0 ** rng.uniform(-9, 5, 20000),
        rng.uniform(-70000, 70000, 5000),
        # exact ties at every binade: (2q + 1) / 2 ulps
        np.concatenate([(2.0 * np.arange(1, 3000) + 1) * 2.0 ** (e - 11) for e in range(-14, 16)]),
        np.array([0.0, -0.0, np.inf, -np.inf, 65504.0, 65519.99, 65520.0, 2.0 ** -24, 2.0 ** -25,
                  2.0 ** -25 * 1.0000001, 2.0 ** -14 * (1 - 2.0 ** -12), 1 + 2.0 ** -11 + 2.0 ** -40]),
    ]
    x = np.concatenate(parts)
    ours = oracle.rn16(x)
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16)
    assert np.array_equal(ours.view(np.uint16), ref.view(np.uint16))
    # a double that would round twice via float32 rounds once here
    assert float(oracle.rn16(np.array([1 + 2.0 ** -11 + 2.0 ** -40]))[0]) == 1.0009765625
    assert np.isnan(oracle.rn16(np.array([np.nan]))[0])


def _rand_half(rng, n, lo=-16, hi=16):
    """binary16 values spread over binades, with subnormals and zeros mixed in."""
    m = rng.integers(0, 1024, n)
    e = rng.integers(lo, hi, n)
    s = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    v = s * np.ldexp(1.0 + m / 1024.0, e)
    sub = rng.random(n) < 0.1
    v[sub] = s[sub] * m[sub] * 2.0 ** -24
    return v.astype(np.float16).astype(np.float64)


def test_fma16_is_exact_rne():
    rng = np.random.default_rng(12)
    n = 6000
    a, b, c = _rand_half(rng, n), _rand_half(rng, n), _rand_half(rng, n)
    # bring c near a*b often so cancellation and ties are exercised
    near = (rng.random(n) < 0.5) & (np.abs(a * b) < 65000)
    c[near] = (-(a * b)[near]).astype(np.float16).astype(np.float64)
    bad = 0
    for i in range(n):
        exact = rne(Fraction(a[i]) * Fraction(b[i]) + Fraction(c[i]), HALF)
        got = oracle.fma16(a[i], b[i], c[i])
        if not (got == exact or (math.isinf(got) and math.isinf(exact) and (got > 0) == (exact > 0))):
            bad += 1
    assert bad == 0


def test_fma32_is_exact_rne():
    rng = np.random.default_rng(13)
    n = 4000
    a = rng.standard_normal(n).astype(np.float32).astype(np.float64)
    b = (rng.standard_normal(n) * 10.0 ** rng.uniform(-6, 6, n)).astype(np.float32).astype(np.float64)
    c = (-(a * b) * (1 + rng.standard_normal(n) * 1e-7)).astype(np.float32).astype(np.float64)
    for i in range(n):
        exact = rne(Fraction(a[i]) * Fraction(b[i]) + Fraction(c[i]), SINGLE)
        assert oracle.fma32(a[i], b[i], c[i]) == exact


# ------------------------------------------------------------------ the tables

def test_theorem_ratio_bounded_all_sizes():
    # Theorem (Sec. III): dual-select keeps |t| <= 1 for every k < N/2
    for m in range(1, 21):
        n = 1 << m
        mult, ratio, path = oracle.table(n, "dual_select")
        assert np.all(np.abs(ratio) <= 1.0)
        # the multiplier is the larger of |cos|, |sin| (Algorithm 1)
        assert np.all(np.abs(mult) >= np.sqrt(0.5) - 1e-15)


def test_linzer_feig_worst_ratio_table1():
    n = int(FACTS["n"])
    tmax, k = oracle.max_ratio(n, "linzer_feig")
    assert k == int(FACTS["lf_tmax_k"])
    assert round(tmax, 1) == FACTS["lf_tmax"]                       # 162.97 prints as 163.0
    assert tmax == pytest.approx(1.0 / math.tan(math.pi / 512), rel=1e-13)
    # the k = 0 entry is the clamped singularity (Sing. = 1): sin(0) -> +1e-7
    mult, ratio, path = oracle.table(n, "linzer_feig")
    assert mult[0] == 1e-7 and ratio[0] == pytest.approx(1e7, rel=1e-15)
    assert int(np.sum(np.abs(oracle.table(n, "linzer_feig")[0]) < 1e-6)) == int(FACTS["lf_sing"])


def test_cosine_near_singularity_table1():
    n = int(FACTS["n"])
    tmax, k = oracle.max_ratio(n, "cosine")
    assert k == int(FACTS["cos_sing_k"]) == n // 4
    assert tmax > FACTS["cos_tmax_lower"]
    mult, _, _ = oracle.table(n, "cosine")
    assert abs(mult[k]) == pytest.approx(FACTS["cos_abs_at_sing"], rel=0.05)


def test_dual_select_max_ratio_table1():
    n = int(FACTS["n"])
    mult, ratio, path = oracle.table(n, "dual_select")
    r = np.abs(ratio)
    tmax = r.max()
    assert round(tmax, 3) == FACTS["ds_tmax"]
    assert tmax == 1.0 - 2.0 ** -53           # FP64 value of tan(pi/4)
    where = set(np.flatnonzero(r == tmax).tolist())
    assert int(FACTS["ds_tmax_k"]) in where and where <= {n // 8, 3 * n // 8}
    # stored in either working precision it is exactly 1.0
    assert np.max(np.abs(ratio.astype(np.float32))) == 1.0
    assert float(np.max(np.abs(oracle.rn16(ratio).astype(np.float64)))) == 1.0
    assert int(FACTS["ds_sing"]) == 0 and np.all(np.isfinite(ratio))


def test_path_split_and_index_rule():
    n = int(FACTS["n"])
    _, _, path = oracle.table(n, "dual_select")
    assert int(np.sum(path == 0)) == int(FACTS["cos_paths"])
    assert int(np.sum(path == 1)) == int(FACTS["sin_paths"])
    for m in range(1, 21):
        nn = 1 << m
        _, _, p = oracle.table(nn, "dual_select")
        k = np.arange(nn // 2)
        rule = np.where((8 * k <= nn) | (8 * k > 3 * nn), 0, 1)
        assert np.array_equal(p, rule), nn


def test_storage_overhead_sec3():
    n = int(FACTS["n"])
    entries = n // 2
    assert entries // 8 == FACTS["flag_bytes"]                     # one bit per twiddle
    assert entries * 2 * 4 == FACTS["table_bytes"]                 # FP32 (mult, ratio)


def test_tables_reconstruct_twiddle():
    for n in (2, 4, 8, 64, 1024, 1 << 16):
        k = np.arange(n // 2)
        w = np.exp(-2j * np.pi * k / n)          # numpy's complex exponential
        for kind in ("dual_select", "cosine", "linzer_feig", "lf_w0_exempt"):
            mult, ratio, path = oracle.table(n, kind)
            eff = np.where(path == 0, mult * (1 + 1j * ratio), mult * (ratio + 1j))
            err = np.abs(eff - w)
            if kind == "linzer_feig":
                assert abs(eff[0] - (1 + 1e-7j)) < 1e-15      # clamped W^0 = 1 + j 1e-7
                err = err[1:]
            if kind == "cosine" and n >= 4:
                err = np.delete(err, n // 4)                  # 6e-17 * 1.6e16 ~ 1 +- ulps
            assert np.all(err < 8e-16), (n, kind, err.max())


def test_table_subsampling_is_exact():
    # theta = -(2 pi k)/N scales exactly by powers of two: T_N[j N/L] == T_L[j]
    big = oracle.table(1 << 14, "dual_select")
    for L in (2, 8, 256, 4096):
        small = oracle.table(L, "dual_select")
        step = (1 << 14) // L
        for a, b in zip(big, small):
            assert np.array_equal(a[::step], b)


# ----------------------------------------------------------- analytic numbers

def test_analytic_bounds_tables_1_2():
    n = int(FACTS["n"])
    assert int(np.log2(n)) == FACTS["passes"]
    u = oracle.UNIT_ROUNDOFF["f16"]
    assert round(u, 6) == FACTS["eps_fp16"] and f"{oracle.UNIT_ROUNDOFF['f32']:.2e}" == "5.96e-08"
    lf_t, _ = oracle.max_ratio(n, "linzer_feig")
    ds_t, _ = oracle.max_ratio(n, "dual_select")
    # with the paper's rounded inputs (163.0, 4.88e-4) the printed values follow exactly
    assert f"{FACTS['lf_tmax'] * FACTS['eps_fp16']:.2e}" == "7.95e-02"
    lf_pb, lf_cum = oracle.analytic_bounds(n, round(lf_t, 1), "f16")
    ds_pb, ds_cum = oracle.analytic_bounds(n, round(ds_t, 3), "f16")
    assert lf_pb == pytest.approx(FACTS["lf_bound_fp16"], rel=2e-3)
    assert ds_pb == pytest.approx(FACTS["ds_bound_fp16"], rel=1e-3)
    assert round(lf_cum, 2) == FACTS["lf_cumulative_fp16"]
    assert round(ds_cum, 5) == FACTS["ds_cumulative_fp16"]
    assert int(lf_cum / ds_cum) == FACTS["improvement"]


# ------------------------------------------------------------- the FP64 result

@pytest.mark.parametrize("n", [2, 4, 8, 16, 64, 128, 256])
def test_fft64_matches_brute_dft(n):
    x = np.random.default_rng(n).standard_normal((3, n, 2))
    d = cplx(oracle.dft64(x))
    f = cplx(oracle.fft64(x))
    assert rel(f, d) < 1e-13


def test_dft64_closed_forms():
    n = 64
    k = np.arange(n)
    for n0 in (0, 1, 5, 63):                      # impulse -> W^{k n0}
        x = np.zeros((1, n, 2)); x[0, n0, 0] = 1.0
        X = cplx(oracle.dft64(x))[0]
        assert np.max(np.abs(X - np.exp(-2j * np.pi * k * n0 / n))) < 1e-13
    x = np.zeros((1, n, 2)); x[0, :, 0] = 0.75; x[0, :, 1] = -0.25   # constant -> cN delta
    X = cplx(oracle.dft64(x))[0]
    assert abs(X[0] - n * (0.75 - 0.25j)) < 1e-12 and np.max(np.abs(X[1:])) < 1e-12
    for f in (1, 7, 33):                           # exp(+j 2 pi f n / N) -> N delta[k - f]
        ph = 2 * np.pi * f * np.arange(n) / n
        x = np.stack([np.cos(ph), np.sin(ph)], -1)[None]
        X = cplx(oracle.dft64(x))[0]
        e = np.zeros(n, complex); e[f] = n
        assert np.max(np.abs(X - e)) < 1e-11


@pytest.mark.parametrize("n", [1 << m for m in range(1, 17, 3)])
def test_fft64_matches_numpy_parseval_linearity(n):
    rng = np.random.default_rng(100 + n)
    x, y = rng.standard_normal((2, 2, n, 2))
    X, Y = cplx(oracle.fft64(x)), cplx(oracle.fft64(y))
    xc = cplx(x)
    assert rel(X, np.fft.fft(xc)) < 1e-13 * max(1, np.log2(n))
    assert np.sum(np.abs(X) ** 2) == pytest.approx(n * np.sum(np.abs(xc) ** 2), rel=1e-12)
    Z = cplx(oracle.fft64(2.5 * x - 0.5 * y))
    assert rel(Z, 2.5 * X - 0.5 * Y) < 1e-13


# ---------------------------------------------------- the six-FMA emulation

@pytest.mark.parametrize("kind", ["dual_select", "cosine", "lf_w0_exempt"])
@pytest.mark.parametrize("n", [2, 4, 8, 32, 256, 1024])
def test_emulation_fp64_is_the_dft(kind, n):
    # the factorisations of Secs. II-B/II-C are exact rewrites of eq. (1)
    x = np.random.default_rng(7 * n).standard_normal((2, n, 2))
    ref = cplx(oracle.dft64(x)) if n <= 256 else np.fft.fft(cplx(x))
    y = cplx(oracle.emulate(x, kind, "f64"))
    tol = 1e-13 if kind != "cosine" or n < 4 else 1e-12
    assert rel(y, ref) < tol


def test_emulation_fp64_linzer_feig_clamp_perturbs():
    # the eps-clamped W^0 = 1 + j 1e-7 is a real perturbation, of order 1e-7 per pass
    n = 256
    x = np.random.default_rng(5).standard_normal((4, n, 2))
    e = rel(cplx(oracle.emulate(x, "linzer_feig", "f64")), cplx(oracle.dft64(x)))
    assert 1e-8 < e < 1e-6


def test_fp16_hand_worked_n4():
    rows = np.loadtxt(os.path.join(GOLDEN, "fp16_n4_worked.txt"))
    x = rows[:, 1:3].astype(np.float16)[None]
    assert np.array_equal(x.astype(np.float64)[0], rows[:, 1:3])     # inputs exact in binary16
    y = oracle.emulate(x, "dual_select", "f16")[0].astype(np.float64)
    assert np.array_equal(y, rows[:, 3:5])


@pytest.mark.parametrize("fname,dtype,npdt", [("fp16_n8_inexact.txt", "f16", np.float16),
                                              ("fp32_n8_inexact.txt", "f32", np.float32)])
def test_hand_worked_n8_inexact_products(fname, dtype, npdt):
    # the W^1 and W^3 entries have m = RN(cos(pi/4)), so every s*m of the last
    # pass is inexact and each of those eight results depends on the FMA being
    # rounded once (Sec. II-B/II-C)
    rows = np.loadtxt(os.path.join(GOLDEN, fname))
    x = rows[:, 1:3].astype(npdt)[None]
    assert np.array_equal(x.astype(np.float64)[0], rows[:, 1:3])     # inputs exact
    y = oracle.emulate(x, "dual_select", dtype)[0].astype(np.float64)
    assert np.array_equal(y, rows[:, 3:5])


def test_fp16_exact_for_small_integers_n4():
    # at N = 4 every dual-select twiddle is exactly 1 or -j in binary16, so small
    # integer inputs transform exactly
    x = np.random.default_rng(3).integers(-50, 50, (20, 4, 2)).astype(np.float16)
    y = oracle.emulate(x, "dual_select", "f16").astype(np.float64)
    assert np.array_equal(cplx(y), np.fft.fft(cplx(x.astype(np.float64))))


def test_fp16_within_cumulative_bound_and_realistic():
    # rel-L2 against FP64 below (1 + u)^m - 1 (eq. (cumulative) with |t| = 1)
    for n, seed in ((1024, 21), (4096, 22)):
        x = np.random.default_rng(seed).uniform(-1, 1, (8, n, 2)).astype(np.float16)
        ref = oracle.fft64(x.astype(np.float64))
        e = oracle.errors(oracle.emulate(x, "dual_select", "f16"), ref)
        bound = (1 + 2.0 ** -11) ** int(np.log2(n)) - 1
        assert e["nonfinite"] == 0
        assert 1e-4 < e["rel_l2"] < bound
        # rounding happens at every FMA: far above the final-rounding-only error
        final_only = oracle.errors(oracle.rn16(ref), ref)["rel_l2"]
        assert e["rel_l2"] > 2 * final_only


def test_fp16_lf_eps_and_cosine_are_nonfinite():
    # RN16(1e7) and RN16(1.6e16) are +inf: the clamped Linzer-Feig and pure-cosine
    # tables are non-finite in binary16 at N = 1024 (Table I "divergent"/163 entries)
    n = 1024
    x = np.random.default_rng(23).uniform(-1, 1, (2, n, 2)).astype(np.float16)
    m, r, _ = oracle.rounded_table(n, "linzer_feig", "f16")
    assert np.isinf(r[0])
    m, r, _ = oracle.rounded_table(n, "cosine", "f16")
    assert np.isinf(r[n // 4])
    ref = oracle.fft64(x.astype(np.float64))
    assert oracle.errors(oracle.emulate(x, "linzer_feig", "f16"), ref)["nonfinite"] == 2 * n
    assert oracle.errors(oracle.emulate(x, "cosine", "f16"), ref)["nonfinite"] > n
    w0 = oracle.errors(oracle.emulate(x, "lf_w0_exempt", "f16"), ref)
    assert w0["nonfinite"] == 0 and w0["rel_l2"] < 5e-3


def test_fp32_error_levels():
    # Sec. V: in FP32 both strategies sit at the ~1e-7 relative-L2 level
    n = 1024
    x = np.random.default_rng(1).standard_normal((16, n, 2)).astype(np.float32)
    ref = oracle.fft64(x.astype(np.float64))
    for kind in ("dual_select", "linzer_feig", "cosine"):
        e = oracle.errors(oracle.emulate(x, kind, "f32"), ref)
        assert e["nonfinite"] == 0
        assert 3e-8 < e["rel_l2"] < 10 * FACTS["fp32_roundtrip_rel_l2"]


# ------------------------------------------- the pins catch planted mistakes

def _pin_checks():
    """The checks a planted mistake must trip (each raises AssertionError)."""
    def dft_check():
        for kind in ("dual_select", "lf_w0_exempt"):
            x = np.random.default_rng(9).standard_normal((2, 64, 2))
            assert rel(cplx(oracle.emulate(x, kind, "f64")), cplx(oracle.dft64(x))) < 1e-13
    def worked_check():
        test_fp16_hand_worked_n4()
    def worked_inexact_f16():
        test_hand_worked_n8_inexact_products("fp16_n8_inexact.txt", "f16", np.float16)
    def worked_inexact_f32():
        test_hand_worked_n8_inexact_products("fp32_n8_inexact.txt", "f32", np.float32)
    def bound_check():
        test_fp16_within_cumulative_bound_and_realistic()
    return [dft_check, worked_check, worked_inexact_f16, worked_inexact_f32, bound_check]


@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5, 6])
def test_planted_mistakes_are_caught(mutant, tmp_path):
    import ctypes
    import subprocess
    so = str(tmp_path / f"mut{mutant}.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    f"-DORC_MUTANT={mutant}", "-o", so, oracle._SRC, "-lm"], check=True)
    saved_lib, saved_path = oracle._lib, oracle._LIB
    try:
        oracle._lib, oracle._LIB = None, so
        caught = 0
        for check in _pin_checks():
            try:
                check()
            except AssertionError:
                caught += 1
        assert caught >= 1, f"mutant {mutant} passed every pin"
    finally:
        oracle._lib, oracle._LIB = saved_lib, saved_path
