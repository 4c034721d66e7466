"""fft_execute_scratch (no device allocation) against fft_execute: same plans,
same inputs, bit-identical outputs, on consecutive calls whose second input
is smaller than the first, for two-pass plans whose intermediate runs through
the library's fixed scratch array in several chunks, and for single-pass
plans (which use no scratch)."""
import numpy as np
import pytest

from paper_2604_00567_amd import binding, inputs
from tests.gpu_util import mismatches

pytestmark = pytest.mark.gpu

SCRATCH = 64 << 20


def _run_both(n, batch, dtype, seed):
    import torch
    x = inputs.uniform(n, batch, seed=seed, dtype=dtype)
    xt = torch.from_numpy(x).to("cuda:0")
    ya = torch.empty_like(xt)
    yb = torch.full_like(xt, float("nan"))
    plan = binding.Plan(n, batch, dtype, "dual_select")
    try:
        plan.execute(xt, ya)
        plan.execute_scratch(xt, yb)
        torch.cuda.synchronize()
        info = plan.info()
    finally:
        plan.close()
    return ya.cpu().numpy(), yb.cpu().numpy(), info


# (n, batch, dtype): the first of each pair is the larger input
CASES = [
    ((1 << 17, 300, "f16"), (1 << 16, 5, "f32")),     # 150 MiB -> 3 chunks; then 2.5 MiB, 1 chunk
    ((1 << 20, 70, "f16"), (1 << 18, 9, "f16")),      # 4 MiB per transform, 5 chunks; then 1 chunk
    ((1 << 20, 20, "f32"), (1 << 15, 33, "f32")),     # 8 MiB per transform, 3 chunks
    ((1 << 10, 4099, "f16"), (1 << 12, 17, "f32")),   # single-pass plans: no scratch
]


@pytest.mark.parametrize("first,second", CASES)
def test_scratch_execute_matches_execute(first, second):
    for k, (n, batch, dtype) in enumerate((first, second)):
        print(f"no-alloc case n={n} batch={batch} dtype={dtype}", flush=True)
        ya, yb, info = _run_both(n, batch, dtype, seed=900 + k + n % 97)
        bad = mismatches(ya, yb)
        assert bad == 0, f"{bad} components differ (n={n}, batch={batch}, {dtype}, {info['config']})"
        two_pass = " | rows:" in info["config"]
        per = n * (4 if dtype == "f16" else 8)
        if two_pass and k == 0:
            assert batch * per > SCRATCH          # the scratch is reused across chunks
        assert np.isfinite(ya).all()


def test_scratch_execute_rejects_bad_arguments():
    import torch
    x = torch.zeros((4, 1 << 17, 2), dtype=torch.float16, device="cuda:0")
    plan = binding.Plan(1 << 17, 4, "f16", "dual_select")
    try:
        with pytest.raises(binding.FFTError) as e:
            binding.fft_execute_scratch(plan.handle, 0, x.data_ptr())
        assert e.value.code == binding.FFT_EINVAL
        with pytest.raises(binding.FFTError) as e:
            binding.fft_execute_scratch(0, x.data_ptr(), x.data_ptr())
        assert e.value.code == binding.FFT_EINVAL
    finally:
        plan.close()
