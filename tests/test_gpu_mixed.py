"""GPU parity of the binary16-storage / binary32-butterfly plans (FFT_F16_F32)
against the oracle's emulation of the same definition (binary16 data widened
exactly, binary32 six-FMA butterflies and table, one rounding of each result
to binary16), bit for bit, for every compiled configuration."""
import numpy as np
import pytest

import oracle
from paper_2604_00567_amd import binding, inputs
from tests.gpu_util import mismatches, run_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("logn", [1, 2, 3, 5, 8, 10, 12, 14, 15, 16, 18, 20])
def test_mixed_all_sizes(logn):
    n = 1 << logn
    batch = 37 if n <= 4096 else max(1, (1 << 19) // n)
    x = inputs.uniform(n, batch, seed=300 + logn, dtype="f16")
    y = run_gpu(x, "f16f32", "dual_select")
    ref = oracle.emulate(x, "dual_select", "f16f32")
    print(f"n={n} batch={batch} mismatches={mismatches(y, ref)}", flush=True)
    assert mismatches(y, ref) == 0


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256, 1024, 4096, 16384, 1 << 15, 1 << 16, 1 << 20])
def test_every_compiled_mixed_configuration(n):
    single, cols, rows = binding.fft_config_count(n, "f16f32")
    assert single + cols * rows > 0
    batch = max(2, min(9, (1 << 18) // n))
    x = inputs.uniform(n, batch, 11, "f16")
    ref = oracle.emulate(x, "dual_select", "f16f32")
    for v in range(single):
        assert mismatches(run_gpu(x, "f16f32", "dual_select", variant=(v, 0, False)), ref) == 0, v
    for a in range(cols):
        for b in range(rows):
            assert mismatches(run_gpu(x, "f16f32", "dual_select", variant=(a, b, True)), ref) == 0, (a, b)


@pytest.mark.parametrize("kind", ["dual_select", "linzer_feig", "cosine", "lf_w0_exempt"])
def test_mixed_every_table_kind_and_inverse(kind):
    import torch
    n, batch = 1024, 8
    x = inputs.uniform(n, batch, 13, "f16")
    assert mismatches(run_gpu(x, "f16f32", kind), oracle.emulate(x, kind, "f16f32")) == 0
    xt = torch.from_numpy(x).to("cuda:0")
    yt = torch.empty_like(xt)
    p = binding.Plan(n, batch, "f16f32", kind, direction="inverse")
    p.execute(xt, yt)
    torch.cuda.synchronize()
    p.close()
    assert mismatches(yt.cpu().numpy(), oracle.emulate(x, kind, "f16f32", inverse=True)) == 0


def test_mixed_accuracy_against_fp64_and_binary16():
    """Binary32 butterflies on binary16 data: the error is the output rounding
    (below 2^-11 relative L2), under that of binary16 butterflies, where the
    Linzer-Feig tables overflow."""
    n, batch = 1024, 64
    x = inputs.uniform(n, batch, 17, "f16")
    exact = oracle.fft64(x.astype(np.float64))
    e_mix = oracle.errors(run_gpu(x, "f16f32", "dual_select"), exact)
    e_f16 = oracle.errors(run_gpu(x, "f16", "dual_select"), exact)
    e_mix_lf = oracle.errors(run_gpu(x, "f16f32", "linzer_feig"), exact)
    assert e_mix["rel_l2"] < 2.0 ** -11 < e_f16["rel_l2"]
    assert e_mix_lf["nonfinite"] == 0                 # binary32 holds the Linzer-Feig ratios


def test_mixed_rejected_where_unsupported():
    with pytest.raises(binding.FFTError):
        binding.Batch([1024, 64], "f16f32")
    with pytest.raises(binding.FFTError):
        binding.fft_serve_slot_create("f16f32", "dual_select", 16, 16, 1, 1 << 20)


@pytest.mark.parametrize("n", [16, 1024])
def test_mixed_special_values(n):
    """Infinities, NaNs, binary16 subnormals, the largest binary16 value and
    -0 through the binary16-storage plans, whose first stage widens its
    operands inside its FMAs (N = 1024) or after staging through LDS (N = 16),
    bit for bit against the oracle (NaN matching NaN)."""
    batch = 8
    x = inputs.uniform(n, batch, 19, "f16")
    flat = x.reshape(-1)
    rng = np.random.default_rng(1)
    idx = rng.choice(flat.size, min(64, flat.size), replace=False)
    flat[idx[:6]] = np.inf
    flat[idx[6:12]] = -np.inf
    flat[idx[12:18]] = np.nan
    flat[idx[18:40]] = np.float16(2.0 ** -24) * rng.integers(-1023, 1024, 22)   # subnormals
    flat[idx[40:48]] = np.float16(65504.0)
    flat[idx[48:]] = np.float16(-0.0)
    x[0] = 0.0                                                                  # an all-zero transform
    x[1] = np.float16(2.0 ** -24)                                               # all smallest subnormal
    x[2] = np.float16(2.0 ** -24) * rng.integers(-1023, 1024, x[2].shape)      # subnormals only
    y = run_gpu(x, "f16f32", "dual_select")
    ref = oracle.emulate(x, "dual_select", "f16f32")
    print(f"n={n} mismatches={mismatches(y, ref)}", flush=True)
    assert mismatches(y, ref) == 0
