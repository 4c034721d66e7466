"""The uneven-batch work list as the library builds it (fft_batch_work_list,
host only), checked for what the two persistent kernels rely on: every
element of every transform is covered exactly once, workspace slices are
disjoint, and every row item is in the second phase while every column item
is in the first."""
import numpy as np
import pytest

from paper_2604_00567_amd import binding, inputs

F = {k: i for i, k in enumerate(binding.WORK_FIELDS)}
# units per item and log2 NU of each configuration id (order of HostBatchCfg)
CFG_LOGNU = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 10, 12, 7, 8, 8, 9, 9, 14]


def classify(it):
    if it[F["phase"]] == 1:
        return "row"
    if it[F["slot"]] >= 0:
        return "col"
    return "small"


def check(sizes, dtype="f16"):
    sizes = np.asarray(sizes, np.int64)
    items, phase0, offs, lst, ws = binding.fft_batch_work_list(sizes, dtype)
    assert np.all(items[:phase0, F["phase"]] == 0) and np.all(items[phase0:, F["phase"]] == 1)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    # binary16 2^16 and 2^15 transforms run whole in the list kernels (the
    # 2^16 list first); larger ones split
    if dtype == "f16":
        listed = (sizes == (1 << 15)) | (sizes == (1 << 16))
        n16 = int(np.sum(sizes == (1 << 16)))
        assert sorted(int(v) for v in lst[:n16]) == sorted(int(v) for v in starts[sizes == (1 << 16)])
        assert sorted(int(v) for v in lst[n16:]) == sorted(int(v) for v in starts[sizes == (1 << 15)])
    else:
        listed = np.zeros(sizes.shape, bool)
    assert sorted(int(v) for v in lst) == sorted(int(v) for v in starts[listed])
    large = (sizes >= (1 << 15)) & ~listed
    assert ws == int(sizes[large].sum())

    # single-unit transforms: each start exactly once, with the class's config
    small_starts = []
    for it in items:
        if classify(it) == "small":
            ln = CFG_LOGNU[it[F["cfg"]]]
            for k in range(it[F["nunits"]]):
                o = int(offs[it[F["first"]] + k])
                small_starts.append(o)
                t = int(np.searchsorted(starts, o))
                assert starts[t] == o and sizes[t] == 1 << ln
    assert sorted(small_starts) == sorted(int(s) for s in starts[sizes < (1 << 15)])

    # large transforms: columns and rows each covered once; waits point back
    by_slot = {}
    ws_slices = {}
    last_col = {}
    for pos, it in enumerate(items):
        kind = classify(it)
        if kind == "col":
            s = it[F["slot"]]
            t = int(np.searchsorted(starts, it[F["in_off"]]))
            assert starts[t] == it[F["in_off"]] and large[t]
            m = int(sizes[t]).bit_length() - 1
            ln = CFG_LOGNU[it[F["cfg"]]]
            assert it[F["log_m"]] == m - ln
            by_slot.setdefault(s, {"t": t, "cols": [], "rows": []})
            assert by_slot[s]["t"] == t
            by_slot[s]["cols"].extend(range(it[F["first"]], it[F["first"]] + it[F["nunits"]]))
            ws_slices.setdefault(s, it[F["out_off"]])
            assert ws_slices[s] == it[F["out_off"]]
            last_col[s] = pos
        elif kind == "row":
            s = it[F["slot"]]
            assert s in last_col, "row item ahead of its transform's column items"
            assert it[F["in_off"]] == ws_slices[s]
            t = by_slot[s]["t"]
            assert it[F["out_off"]] == starts[t]
            m = int(sizes[t]).bit_length() - 1
            assert it[F["log_m"]] == m - CFG_LOGNU[it[F["cfg"]]]
            by_slot[s]["rows"].extend(range(it[F["first"]], it[F["first"]] + it[F["nunits"]]))
            by_slot[s].setdefault("first_row", pos)
            by_slot[s]["nrows"] = 1 << int(it[F["log_m"]])
    for s, d in by_slot.items():
        t = d["t"]
        m = int(sizes[t]).bit_length() - 1
        ncols = 1 << (m - CFG_LOGNU[items[last_col[s]][F["cfg"]]])
        assert sorted(d["cols"]) == list(range(ncols))
        assert sorted(d["rows"]) == list(range(d["nrows"]))
        # the two kernels split the stages: columns x rows points = N
        lc = CFG_LOGNU[items[last_col[s]][F["cfg"]]]
        assert (1 << lc) * ncols == sizes[t] and d["nrows"] * ncols >= 1
    # workspace slices are disjoint and tile [0, ws)
    sl = sorted((ws_slices[s], int(sizes[by_slot[s]["t"]])) for s in by_slot)
    pos = 0
    for a, n in sl:
        assert a == pos
        pos += n
    assert pos == ws
    return items, by_slot, last_col


@pytest.mark.parametrize("dtype", ["f16", "f32"])
def test_work_list_mixed_sizes(dtype):
    sizes = inputs.uneven_sizes(4096, seed=4, log_lo=1, log_hi=18)
    check(sizes, dtype)


def test_work_list_order():
    sizes = inputs.uneven_sizes(600, seed=7, log_lo=6, log_hi=18)
    items, _, _ = check(sizes)
    kinds = [classify(it) for it in items]
    # columns, then whole transforms (largest first), then rows
    order = [k for i, k in enumerate(kinds) if i == 0 or k != kinds[i - 1]]
    assert order == ["col", "small", "row"]
    small_lognu = [CFG_LOGNU[it[F["cfg"]]] for it in items if classify(it) == "small"]
    assert small_lognu == sorted(small_lognu, reverse=True)


def test_work_list_only_small_or_only_large():
    items, phase0, offs, lst, ws = binding.fft_batch_work_list([64] * 100)
    assert phase0 == len(items) and ws == 0 and len(offs) == 100 and len(lst) == 0
    items, phase0, offs, lst, ws = binding.fft_batch_work_list([1 << 17] * 3)
    assert 0 < phase0 < len(items) and ws == 3 << 17 and len(offs) == 0
    check([1 << 17] * 3)
    items, phase0, offs, lst, ws = binding.fft_batch_work_list([1 << 15] * 5, "f16")
    assert len(items) == 0 and ws == 0 and list(lst) == [i << 15 for i in range(5)]
    items, phase0, offs, lst, ws = binding.fft_batch_work_list([1 << 15, 1 << 16, 1 << 15], "f16")
    assert len(items) == 0 and ws == 0 and list(lst) == [1 << 15, 0, 3 << 15]
    items, phase0, offs, lst, ws = binding.fft_batch_work_list([1 << 16] * 3, "f32")
    assert 0 < phase0 < len(items) and ws == 3 << 16 and len(lst) == 0
    check([1 << 16] * 3, "f32")
    items, phase0, offs, lst, ws = binding.fft_batch_work_list([1 << 15] * 5, "f32")
    assert len(items) > 0 and ws == 5 << 15 and len(lst) == 0


def test_work_list_rejects_bad_sizes():
    with pytest.raises(binding.FFTError):
        binding.fft_batch_work_list([1024, 3])
    with pytest.raises(binding.FFTError):
        binding.fft_batch_work_list([1 << 19])
