"""CPU-side checks of the HIP library: it loads, exports every function the
header declares, its host-built tables equal the oracle's bit for bit, and its
argument validation rejects bad requests before touching a GPU."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2604_00567_amd import binding


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(binding.LIB_PATH)
    names = binding.declared_functions()
    assert "fft_plan_create" in names and "fft_execute" in names and "fft_destroy" in names
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("dtype", ["f16", "f32"])
@pytest.mark.parametrize("kind", ["dual_select", "linzer_feig", "cosine", "lf_w0_exempt"])
def test_host_tables_match_oracle(dtype, kind):
    view = np.uint16 if dtype == "f16" else np.uint32
    for m in (1, 2, 3, 5, 8, 10, 12, 16, 20):
        n = 1 << m
        m_lib, r_lib, p_lib = binding.fft_table_build(n, dtype, kind)
        m_orc, r_orc, p_orc = oracle.rounded_table(n, kind, dtype)
        assert np.array_equal(m_lib.view(view), m_orc.view(view)), n
        assert np.array_equal(r_lib.view(view), r_orc.view(view)), n
        assert np.array_equal(p_lib, p_orc.astype(np.uint8)), n


@pytest.mark.parametrize("dtype", ["f16", "f32"])
@pytest.mark.parametrize("kind", ["dual_select", "linzer_feig", "cosine", "lf_w0_exempt"])
def test_host_inverse_tables_match_oracle(dtype, kind):
    view = np.uint16 if dtype == "f16" else np.uint32
    for m in (1, 2, 3, 5, 10, 12, 20):
        n = 1 << m
        m_lib, r_lib, p_lib = binding.fft_table_build(n, dtype, kind, "inverse")
        m_orc, r_orc, p_orc = oracle.rounded_table(n, kind, dtype, inverse=True)
        assert np.array_equal(m_lib.view(view), m_orc.view(view)), n
        assert np.array_equal(r_lib.view(view), r_orc.view(view)), n
        assert np.array_equal(p_lib, p_orc.astype(np.uint8)), n


def test_direction_validation_without_gpu():
    with pytest.raises(binding.FFTError):
        binding.fft_table_build(64, "f16", "dual_select", 0)
    assert "direction" in binding.fft_last_error()
    with pytest.raises(binding.FFTError):
        binding.fft_plan_create_dir(64, 1, "f16", "dual_select", 2)
    assert "direction" in binding.fft_last_error()


def test_dual_select_table_facts_in_storage_precision():
    # Table I: at N = 1024 the stored dual-select ratio peaks at exactly 1.0,
    # the paths split 256 / 256, and the clamped Linzer-Feig entry overflows binary16
    for dtype in ("f16", "f32"):
        m, r, p = binding.fft_table_build(1024, dtype, "dual_select")
        assert float(np.max(np.abs(r.astype(np.float64)))) == 1.0
        assert int(np.sum(p == 0)) == 256 and int(np.sum(p == 1)) == 256
    m, r, p = binding.fft_table_build(1024, "f16", "linzer_feig")
    assert np.isinf(r[0]) and np.all(p == 1)


def test_argument_validation_without_gpu():
    for n in (0, 1, 3, 1000, 1 << 21):
        with pytest.raises(binding.FFTError) as e:
            binding.fft_table_build(n, "f16", "dual_select")
        assert e.value.code == binding.FFT_EINVAL
        with pytest.raises(binding.FFTError):
            binding.fft_plan_create(n, 1, "f16", "dual_select")
        assert "power of two" in binding.fft_last_error()
    with pytest.raises(binding.FFTError):
        binding.fft_plan_create(1024, 0, "f16", "dual_select")
    assert "batch" in binding.fft_last_error()
    with pytest.raises(binding.FFTError):
        binding.fft_table_build(1024, 7, "dual_select")
    with pytest.raises(binding.FFTError):
        binding.fft_table_build(1024, "f16", 9)
    for bad in (3, -1, 7):
        with pytest.raises(binding.FFTError):
            binding.fft_config_count(1024, bad)
        with pytest.raises(binding.FFTError):
            binding.fft_config_count_radix4(1024, bad)
    assert binding.fft_config_count_radix4(1024, "f16f32") == 0
    binding.fft_destroy(None)   # NULL-safe


def test_compiled_configurations_cover_every_size():
    for dtype in ("f16", "f32"):
        for m in range(1, 21):
            single, cols, rows = binding.fft_config_count(1 << m, dtype)
            assert single > 0 or (cols > 0 and rows > 0), (dtype, m)


def test_single_hip_runtime_in_process():
    # the binding loads torch first so the library shares torch's HIP runtime
    with open("/proc/self/maps") as f:
        paths = {line.split()[-1] for line in f if "libamdhip64" in line}
    assert len(paths) == 1, paths


def test_mixed_precision_configurations():
    """Binary16 storage with binary32 butterflies compiles the binary32
    configurations that neither stage nor pipeline: whole transforms up to
    2^15 points (2^15: 64 elements on each of 512 lanes, the exchange in two
    rounds), the two-pass split beyond."""
    for m in range(1, 21):
        n = 1 << m
        s16, c16, r16 = binding.fft_config_count(n, "f32")
        s, c, r = binding.fft_config_count(n, "f16f32")
        assert 0 < s <= s16 if m <= 15 else s == 0
        assert (c > 0 and r > 0) if m >= 12 else True
        assert c <= c16 and r <= r16


def _round(x, dtype):
    return oracle.rn16(x) if dtype == "f16" else np.asarray(x, np.float64).astype(np.float32)


@pytest.mark.parametrize("dtype", ["f16", "f32"])
@pytest.mark.parametrize("kind", ["dual_select", "linzer_feig", "cosine", "lf_w0_exempt"])
@pytest.mark.parametrize("direction", ["forward", "inverse"])
def test_host_radix4_tables_match_oracle(dtype, kind, direction):
    # the radix-4 form reads W^k for k < 3n/4 and, per column, the outer
    # multiplier's choice and rho (computed in FP64, rounded once)
    view = np.uint16 if dtype == "f16" else np.uint32
    inv = direction == "inverse"
    for m in (2, 3, 4, 7, 10, 13, 16, 20):
        n = 1 << m
        m_lib, r_lib, p_lib, rho_lib, sel_lib = binding.fft_table_build_radix4(n, dtype, kind, direction)
        m64, r64, p_orc = oracle.table_count(n, 3 * n // 4, kind, inv)
        rho64, sel_orc = oracle.pairs4(n, kind, inv)
        assert np.array_equal(m_lib.view(view), _round(m64, dtype).view(view)), n
        assert np.array_equal(r_lib.view(view), _round(r64, dtype).view(view)), n
        assert np.array_equal(p_lib, p_orc.astype(np.uint8)), n
        assert np.array_equal(rho_lib.view(view), _round(rho64, dtype).view(view)), n
        assert np.array_equal(sel_lib, sel_orc.astype(np.uint8)), n


def test_radix4_plan_validation_without_gpu():
    # configurations exist for n = 2 .. 2^13 in both storage precisions, none for
    # binary16 storage with binary32 butterflies
    for m in range(1, 14):
        assert binding.fft_config_count_radix4(1 << m, "f16") >= 1
        assert binding.fft_config_count_radix4(1 << m, "f32") >= 1
    assert binding.fft_config_count_radix4(1 << 14, "f16") == 0
    assert binding.fft_config_count_radix4(1024, "f16f32") == 0
    with pytest.raises(binding.FFTError):
        binding.fft_table_build_radix4(2, "f16", "dual_select")
    with pytest.raises(binding.FFTError):
        binding.fft_plan_create_radix4(1024, 1, "f16", "dual_select", 0)
    assert "direction" in binding.fft_last_error()
    with pytest.raises(binding.FFTError):
        binding.fft_plan_create_radix4(1024, 1, "f16f32", "dual_select")
