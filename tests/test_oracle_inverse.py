"""Pins of the oracle's inverse transform (the direction the paper's
round-trip figure of Sec. V implies): library routines and closed forms for
the FP64 inverse, the exact conjugation identity for the emulated butterflies,
the conjugate-table rule, and the binary32 round trip of about 1e-7."""
import numpy as np
import pytest

import oracle
from paper_2604_00567_amd import inputs


def cplx(x):
    x = np.asarray(x, np.float64)
    return x[..., 0] + 1j * x[..., 1]


def inter(z):
    return np.stack([z.real, z.imag], axis=-1)


@pytest.mark.parametrize("n", [2, 4, 8, 32, 64, 256])
def test_inverse_dft_is_numpy_ifft_times_n(n):
    x = inputs.normal(n, 3, 11, "f64")
    got = cplx(oracle.dft64(x, inverse=True))
    ref = np.fft.ifft(cplx(x), axis=-1) * n
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("m", [1, 3, 6, 10, 14, 16])
def test_inverse_fft64_is_numpy_ifft_times_n(m):
    n = 1 << m
    x = inputs.normal(n, 2, 12, "f64")
    got = cplx(oracle.fft64(x, inverse=True))
    ref = np.fft.ifft(cplx(x), axis=-1) * n
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_inverse_closed_forms():
    n = 128
    # inverse of an impulse at k0 is the tone exp(+j 2 pi n k0 / N)
    for k0 in (0, 1, 5, 64, 127):
        X = np.zeros((1, n, 2))
        X[0, k0, 0] = 1.0
        x = cplx(oracle.fft64(X, inverse=True))[0]
        t = np.arange(n)
        assert np.max(np.abs(x - np.exp(2j * np.pi * ((t * k0) % n) / n))) < 1e-13
    # inverse of a constant c is c N at n = 0
    X = np.zeros((1, n, 2))
    X[0, :, 0] = 0.5
    x = cplx(oracle.fft64(X, inverse=True))[0]
    assert abs(x[0] - 0.5 * n) < 1e-12 and np.max(np.abs(x[1:])) < 1e-12


def test_fp64_round_trip_returns_n_times_input():
    for m in (4, 10, 15):
        n = 1 << m
        x = inputs.normal(n, 2, 13, "f64")
        y = oracle.fft64(oracle.fft64(x), inverse=True) / n
        assert np.max(np.abs(y - x)) < 1e-13 * m


@pytest.mark.parametrize("kind", ["dual_select", "linzer_feig", "cosine", "lf_w0_exempt"])
def test_inverse_table_is_the_conjugate_rule(kind):
    # W^{-k} = (w_r, -w_i): cosine path (m, t) -> (m, -t); sine path (m, t) -> (-m, -t),
    # the same path everywhere; Linzer-Feig keeps its +eps clamp at k = 0
    for n in (16, 1024):
        mf, tf, pf = oracle.table(n, kind)
        mi, ti, pi = oracle.table(n, kind, inverse=True)
        assert np.array_equal(pf, pi)
        cos = pf == oracle.PATH_COS
        assert np.array_equal(mi[cos], mf[cos]) and np.array_equal(ti[cos], -tf[cos])
        sin = ~cos
        if kind == "linzer_feig":
            sin[0] = False
            assert mi[0] == mf[0] == oracle.EPS_CLAMP and ti[0] == tf[0]
        assert np.array_equal(mi[sin], -mf[sin]) and np.array_equal(ti[sin], -tf[sin])


@pytest.mark.parametrize("prec", ["f16", "f32"])
@pytest.mark.parametrize("kind", ["dual_select", "lf_w0_exempt"])
def test_emulated_inverse_is_conj_forward_conj(prec, kind):
    # negating an operand is exact, so with the conjugate table every FMA of the
    # inverse is the negation or the copy of one in FFT(conj(x)): bit-identical
    view = np.uint16 if prec == "f16" else np.uint32
    for n in (4, 256, 2048):
        x = inputs.uniform(n, 3, 14, prec)
        a = oracle.emulate(x, kind, prec, inverse=True)
        xc = x.copy()
        xc[..., 1] = -xc[..., 1]
        b = oracle.emulate(xc, kind, prec)
        b[..., 1] = -b[..., 1]
        assert np.array_equal(a.view(view), b.view(view)), n


@pytest.mark.parametrize("kind", ["dual_select", "cosine", "lf_w0_exempt"])
def test_emulated_fp64_inverse_is_the_inverse_dft(kind):
    n = 512
    x = inputs.normal(n, 2, 15, "f64")
    got = cplx(oracle.emulate(x, kind, "f64", inverse=True))
    ref = np.fft.ifft(cplx(x), axis=-1) * n
    tol = 1e-11 if kind != "cosine" else 1e-3     # cosine: |tan| up to 1.6e16 near k = N/4
    assert np.linalg.norm(got - ref) <= tol * np.linalg.norm(ref)


def test_fp32_round_trip_is_about_1e7_as_in_sec_v():
    # Sec. V: in binary32 both strategies give a round trip of about 1e-7 relative L2
    x = inputs.normal(1024, 16, 1, "f32")
    xd = cplx(x)
    for kind in ("dual_select", "linzer_feig"):
        y = cplx(oracle.emulate(oracle.emulate(x, kind, "f32"), kind, "f32", inverse=True)) / 1024
        rel = np.linalg.norm(y - xd) / np.linalg.norm(xd)
        assert 3e-8 < rel < 5e-7, (kind, rel)
