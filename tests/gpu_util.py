"""Helpers for GPU tests: run the HIP path through the C ABI and compare with
the oracle.  Comparisons are bit-exact (NaNs compare equal to NaNs)."""
import numpy as np

from paper_2604_00567_amd import binding


def torch_mod():
    import torch
    return torch


def run_gpu(x: np.ndarray, dtype: str, kind: str, variant=None, inplace: bool = False,
            two_pass: bool = False):
    """x: (batch, n, 2) float16/float32 host array.  Returns the GPU output (host)."""
    torch = torch_mod()
    batch, n, _ = x.shape
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    yt = xt if inplace else torch.empty_like(xt)
    if variant is None and two_pass:
        variant = (0, 0, True)
    plan = binding.Plan(n, batch, dtype, kind, variant)
    try:
        plan.execute(xt, yt)
        torch.cuda.synchronize()
    finally:
        plan.close()
    return yt.cpu().numpy()


def bits(a: np.ndarray) -> np.ndarray:
    return a.view(np.uint16 if a.dtype == np.float16 else np.uint32)


def mismatches(a: np.ndarray, b: np.ndarray) -> int:
    """Number of components whose bit patterns differ (NaN == NaN)."""
    assert a.dtype == b.dtype and a.shape == b.shape
    same = (bits(a) == bits(b)) | (np.isnan(a) & np.isnan(b))
    return int(np.count_nonzero(~same))


def ulp16_diff(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Distance in binary16 units in the last place between finite values."""
    def key(x):
        u = x.view(np.uint16).astype(np.int32)
        return np.where(u & 0x8000, -(u & 0x7FFF), u)
    return np.abs(key(a) - key(b))
