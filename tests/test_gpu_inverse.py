"""GPU parity of the inverse transform (conjugate tables, same kernels) against
the oracle, and the round trip forward -> inverse on the device."""
import numpy as np
import pytest

import oracle
from paper_2604_00567_amd import binding, inputs

from gpu_util import mismatches, torch_mod

pytestmark = pytest.mark.gpu


def run(x, dtype, kind, direction):
    torch = torch_mod()
    batch, n, _ = x.shape
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    yt = torch.empty_like(xt)
    p = binding.Plan(n, batch, dtype, kind, direction=direction)
    try:
        p.execute(xt, yt)
        torch.cuda.synchronize()
    finally:
        p.close()
    return yt.cpu().numpy()


@pytest.mark.parametrize("dtype", ["f16", "f32"])
@pytest.mark.parametrize("logn", [1, 3, 6, 8, 10, 11, 12, 13, 14, 15, 16, 18])
def test_inverse_matches_oracle(dtype, logn):
    n = 1 << logn
    x = inputs.uniform(n, max(2, min(8, (1 << 17) // n)), 21 + logn, dtype)
    ref = oracle.emulate(x, "dual_select", dtype, inverse=True)
    assert mismatches(run(x, dtype, "dual_select", "inverse"), ref) == 0


@pytest.mark.parametrize("dtype", ["f16", "f32"])
@pytest.mark.parametrize("kind", ["dual_select", "linzer_feig", "cosine", "lf_w0_exempt"])
def test_inverse_every_kind(dtype, kind):
    x = inputs.uniform(1024, 6, 22, dtype)
    ref = oracle.emulate(x, kind, dtype, inverse=True)
    assert mismatches(run(x, dtype, kind, "inverse"), ref) == 0


@pytest.mark.parametrize("dtype", ["f16", "f32"])
def test_round_trip_on_device(dtype):
    # forward then inverse on the GPU equals the oracle's round trip bit for bit;
    # binary32 lands near 1e-7 relative L2 (Sec. V)
    x = inputs.normal(1024, 16, 1, dtype)
    y = run(run(x, dtype, "dual_select", "forward"), dtype, "dual_select", "inverse")
    ref = oracle.emulate(oracle.emulate(x, "dual_select", dtype), "dual_select", dtype, inverse=True)
    assert mismatches(y, ref) == 0
    if dtype == "f32":
        xd = x.astype(np.float64)
        rel = np.linalg.norm(y.astype(np.float64) / 1024 - xd) / np.linalg.norm(xd)
        assert 3e-8 < rel < 5e-7


def test_variants_are_forward_only():
    with pytest.raises(binding.FFTError):
        binding.Plan(1024, 2, "f16", "dual_select", variant=(0, 0, False), direction="inverse")
