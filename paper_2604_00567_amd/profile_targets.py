"""Short, fixed workloads to run under a profiler (rocprofv3 --kernel-trace,
--pmc): each executes a plan or batch a few times on synthetic data and exits.

    python -m paper_2604_00567_amd.profile_targets large      # N = 2^15..2^20
    python -m paper_2604_00567_amd.profile_targets batch      # uneven batch
    python -m paper_2604_00567_amd.profile_targets fixed N BATCH DTYPE   # f16, f32, f16f32

Every run starts with three plain 256 MiB device-to-device copies, the
calibration for counter passes (what FETCH_SIZE / WRITE_SIZE read for a copy
of known size).
"""
from __future__ import annotations

import sys

import torch

from . import binding, inputs

TORCH_DTYPE = {"f16": torch.float16, "f32": torch.float32, "f16f32": torch.float16}


def run_fixed(n: int, batch: int, dtype: str, reps: int = 6) -> None:
    x = torch.randn(batch, n, 2, device="cuda").to(TORCH_DTYPE[dtype])
    y = torch.empty_like(x)
    p = binding.Plan(n, batch, dtype, "dual_select")
    print(n, batch, dtype, p.info()["config"], flush=True)
    for _ in range(reps):
        p.execute(x, y)
    torch.cuda.synchronize()
    p.close()


def large() -> None:
    """batch 2^26 / N: binary16 N = 2^15, 2^16 (one kernel each), 2^17, 2^18,
    2^20 (two-pass) and binary32 N = 2^15, 2^16 (two-pass)."""
    for m, dt in ((15, "f16"), (16, "f16"), (17, "f16"), (18, "f16"), (20, "f16"), (15, "f32"),
                  (16, "f32")):
        run_fixed(1 << m, (1 << 26) >> m, dt)
        torch.cuda.empty_cache()


def batch() -> None:
    """4096 transforms, N = 2^U with U uniform over 6..16 (seed 4), binary16."""
    sizes = inputs.uneven_sizes(4096, seed=4)
    x = torch.from_numpy(inputs.packed_uniform(sizes, 4, "f16")).to("cuda:0")
    y = torch.empty_like(x)
    b = binding.Batch(sizes, "f16", "dual_select")
    print(b.info(), flush=True)
    for _ in range(5):
        b.execute(x, y)
    torch.cuda.synchronize()
    b.close()


def calibrate(copies: int = 3, nbytes: int = 256 << 20) -> None:
    """Plain device-to-device copies of `nbytes` (runtime copy kernels)."""
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(copies):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def main(argv) -> int:
    torch.cuda.set_stream(torch.cuda.Stream())
    calibrate()
    if argv[:1] == ["large"]:
        large()
    elif argv[:1] == ["batch"]:
        batch()
    elif argv[:1] == ["fixed"] and len(argv) == 4:
        run_fixed(int(argv[1]), int(argv[2]), argv[3])
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
