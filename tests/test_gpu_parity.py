"""GPU parity: the HIP path against the oracle's emulation of the same radix-2
Stockham pass order with six-FMA butterflies, element by element.

The bar is bit equality (NaN matching NaN): every GPU butterfly computes the
same FMAs, on the same operands, with the same table entry, as the emulation.
The tolerances the method states (1 binary16 ulp per element per pass; 1e-6
relative L2 in binary32 at N = 1024) are asserted as well, so a failure of
bit equality that stays inside them is reported separately.
"""
import numpy as np
import pytest

import oracle
from paper_2604_00567_amd import binding, inputs
from tests.gpu_util import mismatches, run_gpu, ulp16_diff

pytestmark = pytest.mark.gpu


def describe_mismatch(y, ref, limit=6):
    bad = np.argwhere(~((y.view(np.uint16 if y.dtype == np.float16 else np.uint32) ==
                         ref.view(np.uint16 if ref.dtype == np.float16 else np.uint32)) |
                        (np.isnan(y) & np.isnan(ref))))
    return "; ".join(f"{tuple(i)}: gpu={y[tuple(i)]!r} oracle={ref[tuple(i)]!r}" for i in bad[:limit])


def check_f16(y, ref, n):
    print(f"check n={n} shape={y.shape} mismatches={mismatches(y, ref)} "
          f"{describe_mismatch(y, ref)}", flush=True)
    finite = np.isfinite(ref) & np.isfinite(y)
    m = int(np.log2(n))
    assert np.all(np.isnan(y) == np.isnan(ref))
    assert np.all(ulp16_diff(y[finite], ref[finite]) <= m)      # stated tolerance
    assert mismatches(y, ref) == 0                                # design: bit-exact


def check_f32(y, ref):
    e = oracle.errors(y, ref.astype(np.float64))
    assert e["nonfinite"] == 0 or np.all(np.isnan(y) == np.isnan(ref))
    if e["nonfinite"] == 0:
        assert e["rel_l2"] <= 1e-6                                # stated tolerance
    assert mismatches(y, ref) == 0                                # design: bit-exact


@pytest.mark.parametrize("logn", list(range(1, 17)))
def test_fp16_dual_select_all_sizes(logn):
    n = 1 << logn
    batch = 37 if n <= 4096 else 3              # ragged against every units-per-workgroup
    x = inputs.uniform(n, batch, seed=100 + logn, dtype="f16")
    y = run_gpu(x, "f16", "dual_select")
    check_f16(y, oracle.emulate(x, "dual_select", "f16"), n)


@pytest.mark.parametrize("logn", list(range(1, 17)))
def test_fp32_dual_select_all_sizes(logn):
    n = 1 << logn
    batch = 37 if n <= 4096 else 3
    x = inputs.normal(n, batch, seed=200 + logn, dtype="f32")
    y = run_gpu(x, "f32", "dual_select")
    check_f32(y, oracle.emulate(x, "dual_select", "f32"))


@pytest.mark.parametrize("dtype", ["f16", "f32"])
@pytest.mark.parametrize("kind", ["dual_select", "linzer_feig", "cosine", "lf_w0_exempt"])
def test_every_table_kind_n1024(dtype, kind):
    n, batch = 1024, 16
    x = (inputs.uniform(n, batch, 3, "f16") if dtype == "f16" else inputs.normal(n, batch, 1, "f32"))
    y = run_gpu(x, dtype, kind)
    ref = oracle.emulate(x, kind, dtype)
    assert mismatches(y, ref) == 0
    if dtype == "f16" and kind in ("linzer_feig", "cosine"):
        # RN16(1e7) and RN16(1.6e16) are +inf: the outputs are non-finite, as emulated
        assert not np.all(np.isfinite(y))


@pytest.mark.parametrize("dtype", ["f16", "f32"])
@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384, 1 << 15, 1 << 16,
                               1 << 18, 1 << 20])
def test_every_compiled_configuration(dtype, n):
    """Every single-kernel configuration, and every column x row pair of the
    two-pass schedule, bit for bit against the oracle."""
    single, cols, rows = binding.fft_config_count(n, dtype)
    batch = max(2, min(9, (1 << 18) // n))
    x = inputs.uniform(n, batch, 7, dtype)
    ref = oracle.emulate(x, "dual_select", dtype)
    for v in range(single):
        assert mismatches(run_gpu(x, dtype, "dual_select", variant=(v, 0, False)), ref) == 0, v
    for a in range(cols):
        for b in range(rows):
            y = run_gpu(x, dtype, "dual_select", variant=(a, b, True))
            assert mismatches(y, ref) == 0, (a, b)


@pytest.mark.parametrize("dtype", ["f16", "f32"])
def test_in_place(dtype):
    for n in (1024, 1 << 15):
        x = inputs.uniform(n, 5, 8, dtype)
        y = run_gpu(x, dtype, "dual_select", inplace=True)
        assert mismatches(y, oracle.emulate(x, "dual_select", dtype)) == 0


@pytest.mark.parametrize("dtype", ["f16", "f32"])
def test_largest_size(dtype):
    n = 1 << 20
    x = inputs.tones(n, 2, 33, dtype)
    y = run_gpu(x, dtype, "dual_select")
    assert mismatches(y, oracle.emulate(x, "dual_select", dtype)) == 0


def test_special_values_fp16():
    n, batch = 1024, 8
    x = inputs.uniform(n, batch, 9, "f16")
    flat = x.reshape(-1)
    rng = np.random.default_rng(0)
    idx = rng.choice(flat.size, 64, replace=False)
    flat[idx[:8]] = np.inf
    flat[idx[8:16]] = -np.inf
    flat[idx[16:24]] = np.nan
    flat[idx[24:40]] = np.float16(2.0 ** -24) * rng.integers(-1023, 1024, 16)   # subnormals
    flat[idx[40:48]] = np.float16(65504.0)
    flat[idx[48:64]] = np.float16(-0.0)
    x[0] = 0.0                                                                  # an all-zero transform
    x[1] = np.float16(2.0 ** -24)                                               # all smallest subnormal
    y = run_gpu(x, "f16", "dual_select")
    assert mismatches(y, oracle.emulate(x, "dual_select", "f16")) == 0


def test_fp32_subnormals_kept():
    n, batch = 256, 4
    x = (inputs.normal(n, batch, 10, "f32") * np.float32(1e-39)).astype(np.float32)
    y = run_gpu(x, "f32", "dual_select")
    assert mismatches(y, oracle.emulate(x, "dual_select", "f32")) == 0
    assert np.any(y != 0)


def test_batch_one_and_smallest_n():
    for n in (2, 4, 1024):
        x = inputs.uniform(n, 1, 11, "f16")
        assert mismatches(run_gpu(x, "f16", "dual_select"), oracle.emulate(x, "dual_select", "f16")) == 0


@pytest.mark.parametrize("n,batch,samples", [(1024, 65536, 48), (4096, 16384, 24)])
def test_full_size_sampled(n, batch, samples):
    """Batched FP16 fixed-size workload at full size; sampled transforms are
    checked one by one against the emulation, all of them against FP64 bounds."""
    x = inputs.uniform(n, batch, seed=2, dtype="f16")
    y = run_gpu(x, "f16", "dual_select")
    pick = np.random.default_rng(5).choice(batch, samples, replace=False)
    pick = np.concatenate([pick, [0, batch - 1]])
    ref = oracle.emulate(x[pick], "dual_select", "f16")
    assert mismatches(y[pick], ref) == 0
    e = oracle.errors(y[pick], oracle.fft64(x[pick].astype(np.float64)))
    assert e["nonfinite"] == 0 and e["rel_l2"] < (1 + 2.0 ** -11) ** int(np.log2(n)) - 1
    assert np.all(np.isfinite(y))


@pytest.mark.parametrize("n,dtype,two_pass", [(1024, "f16", False), (1 << 16, "f16", True),
                                              (4096, "f32", False)])
def test_more_than_2e31_elements(n, dtype, two_pass):
    """One launch over 2^31 + complex elements (8-16 GiB each way): every
    element offset needs 64 bits.  A small distinct block is tiled over the
    whole batch on the device; sampled transforms (the last ones included) are
    compared with the oracle."""
    torch = pytest.importorskip("torch")
    total = (1 << 31) + (1 << 20)
    batch = total // n
    distinct = 32
    x0 = inputs.uniform(n, distinct, 17, dtype)
    xt = torch.from_numpy(x0).to("cuda:0").repeat((batch + distinct - 1) // distinct, 1, 1)[:batch]
    yt = torch.empty_like(xt)
    plan = binding.Plan(n, batch, dtype, "dual_select", variant=(0, 0, True) if two_pass else None)
    try:
        plan.execute(xt, yt)
        torch.cuda.synchronize()
    finally:
        plan.close()
    ref = oracle.emulate(x0, "dual_select", dtype)
    for b in (0, 1, batch // 2, batch - 2, batch - 1):
        assert mismatches(yt[b].cpu().numpy()[None], ref[b % distinct][None]) == 0, b
    del xt, yt
    torch.cuda.empty_cache()


def test_argument_errors():
    torch = pytest.importorskip("torch")
    n, batch = 1024, 4
    plan = binding.fft_plan_create(n, batch, "f16", "dual_select")
    try:
        x = torch.zeros((batch * n * 2 + 8,), dtype=torch.float16, device="cuda:0")
        base = x.data_ptr()
        with pytest.raises(binding.FFTError) as e:
            binding.fft_execute(plan, base + 2, base + 2)          # misaligned
        assert e.value.code == binding.FFT_EINVAL
        with pytest.raises(binding.FFTError) as e:
            binding.fft_execute(plan, base, base + 8)              # partial overlap
        assert e.value.code == binding.FFT_EINVAL
        with pytest.raises(binding.FFTError) as e:
            binding.fft_execute(plan, 0, base)
        assert e.value.code == binding.FFT_EINVAL
    finally:
        binding.fft_destroy(plan)
    for bad in ((1000, 1), (1 << 21, 1), (1024, 0)):
        with pytest.raises(binding.FFTError):
            binding.fft_plan_create(bad[0], bad[1], "f16", "dual_select")


@pytest.mark.parametrize("dtype", ["f16", "f32"])
def test_unaligned_pointers_use_plain_kernel(dtype):
    """Element-aligned but not 16-byte aligned data takes the unstaged kernel."""
    torch = pytest.importorskip("torch")
    n, batch = 1024, 6
    x = inputs.uniform(n, batch, 12, dtype)
    eb = 4 if dtype == "f16" else 8
    tdt = torch.float16 if dtype == "f16" else torch.float32
    per = eb // (2 if dtype == "f16" else 4)          # storage values per element (2)
    buf_in = torch.zeros(n * batch * 2 + 16, dtype=tdt, device="cuda:0")
    buf_out = torch.zeros_like(buf_in)
    off = per                                          # one element: 4 or 8 bytes
    buf_in[off:off + n * batch * 2] = torch.from_numpy(x.reshape(-1)).to("cuda:0")
    plan = binding.fft_plan_create(n, batch, dtype, "dual_select")
    try:
        binding.fft_execute(plan, buf_in.data_ptr() + off * buf_in.element_size(),
                            buf_out.data_ptr() + off * buf_out.element_size(),
                            torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    finally:
        binding.fft_destroy(plan)
    y = buf_out[off:off + n * batch * 2].cpu().numpy().reshape(batch, n, 2)
    assert mismatches(y, oracle.emulate(x, "dual_select", dtype)) == 0


def pipelined_sizes():
    """log2 N of the whole-transform configurations with PIPE = 1 in the
    configuration list (the sizes the pipelined test has work for)."""
    import os
    import re
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2604_00567_amd", "csrc", "configs.inc")
    out = set()
    for line in open(path):
        m = re.match(r"\s*CFG[UE]?\(MODE_SMALL,\s*(\d+)," + r"\s*\d+," * 7 + r"\s*(\d+)", line)
        if m and int(m.group(2)) == 1:
            out.add(int(m.group(1)))
    return sorted(out)


@pytest.mark.parametrize("dtype", ["f16", "f32"])
@pytest.mark.parametrize("logn", pipelined_sizes())
def test_pipelined_configurations_over_many_blocks(dtype, logn):
    """Every pipelined (persistent, two register sets) configuration over a
    batch of several blocks per resident workgroup, so that both register sets
    and the prefetch of a next block run, with a ragged last block; sampled
    transforms (first, last, and random ones) against the oracle."""
    torch = pytest.importorskip("torch")
    n = 1 << logn
    single, _, _ = binding.fft_config_count(n, dtype)
    elem = 4 if dtype == "f16" else 8
    batch = (1 << 27) // (n * elem) - 3
    pipelined = []
    for v in range(single):
        p = binding.Plan(n, batch, dtype, "dual_select", variant=(v, 0, False))
        try:
            if "pipe=1" in p.info()["config"]:
                pipelined.append((v, p.info()["config"]))
        finally:
            p.close()
    if not pipelined:
        pytest.skip("no pipelined configuration at this size")
    x0 = inputs.uniform(n, 64, 23, dtype)
    ref0 = oracle.emulate(x0, "dual_select", dtype)
    xt = torch.from_numpy(x0).to("cuda:0").repeat((batch + 63) // 64, 1, 1)[:batch].contiguous()
    pick = np.concatenate([[0, 1, batch // 2, batch - 2, batch - 1],
                           np.random.default_rng(logn).choice(batch, 11, replace=False)])
    for v, cfg in pipelined:
        yt = torch.full_like(xt, float("nan"))
        p = binding.Plan(n, batch, dtype, "dual_select", variant=(v, 0, False))
        try:
            p.execute(xt, yt)
            torch.cuda.synchronize()
        finally:
            p.close()
        y = yt[torch.from_numpy(pick)].cpu().numpy()
        print(f"pipelined n={n} {dtype} batch={batch} variant={v} {cfg}", flush=True)
        assert mismatches(y, ref0[pick % 64]) == 0, (v, cfg)
        del yt
    del xt
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,dtype", [(1 << 17, "f16"), (1 << 20, "f16"), (1 << 16, "f32"),
                                     (1 << 20, "f32")])
def test_large_n_sweep_full_size_sampled(n, dtype):
    """Large-N sweep at its full size (batch * N = 2^26 elements, tone inputs)
    through the library's default (tuned) two-pass plan: a block of distinct
    transforms tiled over the batch on the device, sampled transforms (the
    first two, the last, and the two on either side of the middle, which is a
    boundary between 128 MiB workspace chunks at every size here) bit for bit
    against the oracle."""
    torch = pytest.importorskip("torch")
    batch = (1 << 26) // n
    distinct = 4
    x0 = inputs.tones(n, distinct, 19, dtype)
    xt = torch.from_numpy(x0).to("cuda:0").repeat(batch // distinct, 1, 1).contiguous()
    yt = torch.empty_like(xt)
    plan = binding.Plan(n, batch, dtype, "dual_select")
    try:
        cfg = plan.info()["config"]
        plan.execute(xt, yt)
        torch.cuda.synchronize()
    finally:
        plan.close()
    print(f"large-N sweep n={n} {dtype} batch={batch} {cfg}", flush=True)
    assert " | " in cfg                                   # the two-pass schedule
    ref = oracle.emulate(x0, "dual_select", dtype)
    for b in sorted({0, 1, batch // 2 - 1, batch // 2, batch - 1}):
        assert mismatches(yt[b].cpu().numpy()[None], ref[b % distinct][None]) == 0, b
    del xt, yt
    torch.cuda.empty_cache()
