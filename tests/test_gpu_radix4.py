"""GPU parity of the radix-4 form (Sec. VI, generality): every compiled radix-4
configuration against the oracle's radix-4 emulation (canonical radix-4
Stockham order, 22 FMAs per butterfly, each rounded once), element by element,
through the C ABI.  The bar is bit equality (NaN matching NaN), as for the
radix-2 path.  Also: every table kind, the inverse, and the binary16 error of
the radix-4 form against the FP64 FFT beside the radix-2 path's."""
import numpy as np
import pytest

import oracle
from paper_2604_00567_amd import binding, inputs
from tests.gpu_util import mismatches

pytestmark = pytest.mark.gpu

KINDS = ("dual_select", "linzer_feig", "cosine", "lf_w0_exempt")


def run_radix4(x, dtype, kind, variant=-1, direction="forward"):
    import torch
    batch, n, _ = x.shape
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    yt = torch.empty_like(xt)
    plan = binding.Plan(n, batch, dtype, kind, variant=variant, direction=direction, radix=4)
    try:
        plan.execute(xt, yt)
        torch.cuda.synchronize()
        cfg = plan.info()["config"]
    finally:
        plan.close()
    assert ",radix4" in cfg
    return yt.cpu().numpy(), cfg


def gen(n, batch, dtype, seed):
    return inputs.uniform(n, batch, seed=seed, dtype=dtype) if dtype == "f16" else \
        inputs.normal(n, batch, seed=seed, dtype=dtype)


CASES = [(1 << m, dt, v) for dt in ("f16", "f32") for m in range(1, 14)
         for v in range(binding.fft_config_count_radix4(1 << m, dt))]


@pytest.mark.parametrize("n,dtype,variant", CASES)
def test_every_radix4_configuration(n, dtype, variant):
    batch = 37 if n <= 1024 else 5             # ragged against the units per workgroup
    x = gen(n, batch, dtype, seed=700 + n % 251 + variant)
    print(f"radix4 n={n} dtype={dtype} variant={variant}", flush=True)
    y, cfg = run_radix4(x, dtype, "dual_select", variant)
    ref = oracle.emulate4(x, "dual_select", dtype)
    assert mismatches(y, ref) == 0, cfg


@pytest.mark.parametrize("dtype", ["f16", "f32"])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("direction", ["forward", "inverse"])
def test_radix4_kinds_and_directions(dtype, kind, direction):
    for n in (8, 64, 2048, 4096):
        x = gen(n, 9, dtype, seed=800 + n % 97)
        y, cfg = run_radix4(x, dtype, kind, direction=direction)
        ref = oracle.emulate4(x, kind, dtype, inverse=direction == "inverse")
        assert mismatches(y, ref) == 0, (n, cfg)


def test_radix4_binary16_error_beside_radix2():
    # N = 1024 binary16 uniform[-1, 1): both forms within the cumulative bound
    # (1 + 2^-11)^10 - 1 of the radix-2 dual-select analysis; the radix-4
    # butterfly keeps every ratio (t and rho) at most 1 in magnitude
    import torch
    n, batch = 1024, 64
    x = inputs.uniform(n, batch, seed=2, dtype="f16")
    y4, _ = run_radix4(x, "f16", "dual_select")
    xt = torch.from_numpy(x).to("cuda:0")
    yt = torch.empty_like(xt)
    p = binding.Plan(n, batch, "f16", "dual_select")
    p.execute(xt, yt)
    torch.cuda.synchronize()
    p.close()
    y2 = yt.cpu().numpy()
    ref = oracle.fft64(x.astype(np.float64))
    e4 = oracle.errors(y4, ref)
    e2 = oracle.errors(y2, ref)
    bound = (1 + 2.0 ** -11) ** 10 - 1
    print(f"radix-4 {e4}  radix-2 {e2}", flush=True)
    assert e4["nonfinite"] == 0 and e2["nonfinite"] == 0
    assert e4["rel_l2"] <= bound and e2["rel_l2"] <= bound
