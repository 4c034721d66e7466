"""GPU tests of the autotuners: every candidate is bit-identical to the
default configuration, the recorded choice is what later plans use, and the
record file round-trips."""
import os

import numpy as np
import pytest

from paper_2604_00567_amd import binding

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,dtype", [(1024, "f16"), (4096, "f16"), (1024, "f32"), (1 << 15, "f16")])
def test_tune_records_fastest_bit_exact(n, dtype, tmp_path):
    rep = binding.fft_tune(n, max(1, (1 << 22) // n), dtype, "dual_select", reps=5)
    assert rep and all(c["bit_exact"] for c in rep), rep
    timed = [c for c in rep if c["GBs"] > 0]
    best = max(timed, key=lambda c: c["GBs"])
    choice = binding.fft_tuned_choice(n, dtype)
    assert choice is not None and list(choice) == [best["variant"][0], best["variant"][1],
                                                   bool(best["variant"][2])]
    p = binding.Plan(n, max(1, (1 << 22) // n), dtype, "dual_select")
    try:
        assert p.info()["config"].split(" | ")[0] == best["config"].split(" | ")[0]
    finally:
        p.close()


@pytest.mark.parametrize("dtype", ["f16", "f32", "f16f32"])
def test_small_batch_takes_one_transform_per_workgroup(dtype):
    """A batch too small to give every compute unit a workgroup under the
    tuned configuration runs one transform per workgroup (where the size has
    such a configuration), with the same results bit for bit."""
    import oracle
    from paper_2604_00567_amd import inputs
    from tests.gpu_util import mismatches, run_gpu
    n = 1024
    small = binding.Plan(n, 16, dtype, "dual_select")
    large = binding.Plan(n, 1 << 16, dtype, "dual_select")
    try:
        assert ",upw=1," in small.info()["config"] and "pipe=0" in small.info()["config"]
        assert ",upw=1," not in large.info()["config"]
    finally:
        small.close()
        large.close()
    x = inputs.normal(n, 16, 1, "f16" if dtype != "f32" else "f32")
    ref = oracle.emulate(x, "dual_select", dtype)
    assert mismatches(run_gpu(x, dtype, "dual_select"), ref) == 0


def test_batch_tune_returns_choices():
    a, b = binding.fft_batch_tune("f16", "dual_select", reps=3)
    assert a in (0, 1) and b in (0, 1)


def test_batch_tune_classes_returns_choices():
    alt = binding.fft_batch_tune_classes("f16", "dual_select", reps=2)
    assert len(alt) == 15 and set(alt) <= {0, 1}
    assert all(alt[m] == 0 for m in list(range(0, 7)) + [13, 14])   # classes without an alternative
