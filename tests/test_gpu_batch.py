"""GPU parity of the uneven-size batch (one persistent-kernel launch replayed
from a HIP graph): every transform against the oracle's emulation, and equal
bit for bit to the same transform computed by a regular plan."""
import numpy as np
import pytest

import oracle
from paper_2604_00567_amd import binding, inputs
from tests.gpu_util import mismatches, run_gpu

pytestmark = pytest.mark.gpu


def split(y, sizes):
    out, o = [], 0
    for n in sizes:
        out.append(y[o:o + n])
        o += n
    return out


def run_batch(sizes, x, dtype, replays=1, choice=None, inplace=False):
    import torch
    b = binding.Batch(sizes, dtype, "dual_select", choice)
    try:
        xt = torch.from_numpy(x).to("cuda:0")
        yt = xt if inplace else torch.empty_like(xt)
        outs = []
        for r in range(replays):
            b.execute(xt, yt)
            torch.cuda.synchronize()
            outs.append(yt.cpu().numpy().copy())
            # eager work between replays, on the same stream
            z = torch.randn(1 << 20, device="cuda:0")
            z.mul_(2.0).sum().item()
        return outs, b.info()
    finally:
        b.close()


def check_all(sizes, x, y, dtype):
    xs, ys = split(x, sizes), split(y, sizes)
    by_n = {}
    for i, n in enumerate(sizes):
        by_n.setdefault(int(n), []).append(i)
    for n, idx in by_n.items():
        xb = np.stack([xs[i] for i in idx])
        yb = np.stack([ys[i] for i in idx])
        assert mismatches(yb, oracle.emulate(xb, "dual_select", dtype)) == 0, n


@pytest.mark.parametrize("dtype", ["f16", "f32"])
def test_every_size_in_one_launch(dtype):
    # every size the batch accepts, 2 .. 2^18: whole-transform items, the
    # binary16 2^15/2^16 list kernels and the column/row split of the larger
    # sizes (binary16 2^17-2^18, binary32 2^15-2^18)
    sizes = np.array([1 << m for m in range(1, 19)] * 3 + [1024] * 20 + [64] * 40, dtype=np.int64)
    np.random.default_rng(1).shuffle(sizes)
    x = inputs.packed_uniform(sizes, 41, dtype)
    (y,), info = run_batch(sizes, x, dtype)
    assert info["items"] > 0 and info["grid"] > 0
    check_all(sizes, x, y, dtype)


def test_graph_replays_and_new_buffers():
    import torch
    sizes = inputs.uneven_sizes(300, seed=5)
    x1 = inputs.packed_uniform(sizes, 51, "f16")
    x2 = inputs.packed_uniform(sizes, 52, "f16")
    b = binding.Batch(sizes, "f16")
    try:
        a1 = torch.from_numpy(x1).to("cuda:0")
        a2 = torch.from_numpy(x2).to("cuda:0")
        y1, y2 = torch.empty_like(a1), torch.empty_like(a2)
        res = []
        for k in range(4):                       # replays, alternating buffers
            src, dst = (a1, y1) if k % 2 == 0 else (a2, y2)
            dst.zero_()
            b.execute(src, dst)
            torch.cuda.synchronize()
            res.append(dst.cpu().numpy().copy())
            torch.randn(4096, device="cuda:0").sum().item()   # eager work in between
        assert mismatches(res[0], res[2]) == 0 and mismatches(res[1], res[3]) == 0
    finally:
        b.close()
    check_all(sizes, x1, res[0], "f16")
    check_all(sizes, x2, res[1], "f16")


def test_uneven_full_workload_sampled():
    """4096 transforms, N = 2^U with U uniform over 6..16, binary16, in place
    and out of place; sampled transforms against the emulation and against a
    regular plan of the same size."""
    sizes = inputs.uneven_sizes(4096, seed=4)
    x = inputs.packed_uniform(sizes, 4, "f16")
    (y,), info = run_batch(sizes, x, "f16")
    (yi,), _ = run_batch(sizes, x, "f16", inplace=True)
    assert mismatches(y, yi) == 0
    xs, ys = split(x, sizes), split(y, sizes)
    rng = np.random.default_rng(7)
    for m in range(6, 17):
        idx = np.flatnonzero(sizes == (1 << m))
        pick = rng.choice(idx, min(3, idx.size), replace=False)
        xb = np.stack([xs[i] for i in pick])
        yb = np.stack([ys[i] for i in pick])
        assert mismatches(yb, oracle.emulate(xb, "dual_select", "f16")) == 0, m
        assert mismatches(yb, run_gpu(xb, "f16", "dual_select")) == 0, m


@pytest.mark.parametrize("choice", [(0, 0), (1, 1)])
def test_tuned_alternatives_bit_identical(choice):
    sizes = np.array([1024] * 37 + [4096] * 11, dtype=np.int64)
    x = inputs.packed_uniform(sizes, 61, "f16")
    (y,), _ = run_batch(sizes, x, "f16", choice=choice)
    check_all(sizes, x, y, "f16")


@pytest.mark.parametrize("dtype", ["f16", "f32"])
def test_class_alternatives_bit_identical(dtype):
    # every class with an alternative configuration (2^7 .. 2^12) takes it,
    # ragged against each configuration's units per workgroup; the oracle decides
    alt = [0] * 15
    for m in range(7, 13):
        alt[m] = 1
    sizes = np.array([128] * 35 + [256] * 19 + [512] * 21 + [1024] * 9 + [2048] * 7 + [4096] * 5 + [64] * 3,
                     dtype=np.int64)
    x = inputs.packed_uniform(sizes, 62, dtype)
    (y,), _ = run_batch(sizes, x, dtype, choice=alt)
    check_all(sizes, x, y, dtype)


def test_batch_argument_errors():
    for bad in ([3], [1 << 19], [0], []):
        with pytest.raises(binding.FFTError):
            binding.fft_batch_create(np.array(bad, dtype=np.int64), "f16", "dual_select")
