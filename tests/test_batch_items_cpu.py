"""CPU model of the uneven-batch work list (mirrors batch.cpp's ordering rule)
checking the properties the persistent kernel relies on: every element is
covered exactly once, workspace slices are disjoint, and every row item only
waits on column items queued before it."""
import numpy as np

from paper_2604_00567_amd import inputs

UPW_SMALL = {1: 256, 2: 256, 3: 256, 4: 64, 5: 64, 6: 32, 7: 32, 8: 16, 9: 16, 10: 8, 11: 4,
             12: 1, 13: 1}
SPLIT = {14: (7, 32, 7, 32, 7), 15: (8, 16, 7, 32, 8), 16: (8, 16, 8, 16, 8)}  # (lognu_c, upw_c, lognu_r, upw_r, ...)


def build(sizes):
    cols, rows, small = [], [], []
    ws, slot, offset = 0, 0, 0
    offs = []
    by_class = {}
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    for t, n in enumerate(sizes):
        m = int(n).bit_length() - 1
        if m <= 13:
            by_class.setdefault(m, []).append(int(starts[t]))
            continue
        lnc, uc, lnr, ur, _ = SPLIT[m]
        lm_c, lm_r = m - lnc, m - lnr
        citems = 0
        for r0 in range(0, 1 << lm_c, uc):
            cols.append(("c", t, r0, min(uc, (1 << lm_c) - r0), slot, ws))
            citems += 1
        for q0 in range(0, 1 << lm_r, ur):
            rows.append(("r", t, q0, min(ur, (1 << lm_r) - q0), slot, citems, ws))
        ws += int(n)
        slot += 1
    for m in sorted(by_class, reverse=True):
        v = by_class[m]
        for i in range(0, len(v), UPW_SMALL[m]):
            small.append(("s", m, len(offs), min(UPW_SMALL[m], len(v) - i)))
            offs.extend(v[i:i + UPW_SMALL[m]])
    return cols + small + rows, offs, ws


def test_work_list_properties():
    sizes = inputs.uneven_sizes(4096, seed=4, log_lo=1, log_hi=16)
    items, offs, ws = build(sizes)
    # single-unit transforms appear exactly once
    small_starts = sorted(offs)
    expect = sorted(int(s) for s, n in zip(np.concatenate([[0], np.cumsum(sizes)[:-1]]), sizes)
                    if n <= 1 << 13)
    assert small_starts == expect
    # every residue / row of a big transform exactly once; waits point backwards
    seen_cols, done_cols = {}, {}
    for pos, it in enumerate(items):
        if it[0] == "c":
            _, t, r0, nu, slot, w = it
            seen_cols.setdefault(t, set()).update(range(r0, r0 + nu))
            done_cols[slot] = done_cols.get(slot, 0) + 1
        elif it[0] == "r":
            _, t, q0, nu, slot, need, w = it
            assert done_cols.get(slot, 0) == need, "row item queued before its column items"
    for t, s in seen_cols.items():
        m = int(sizes[t]).bit_length() - 1
        assert s == set(range(1 << (m - SPLIT[m][0])))
    assert ws == int(np.sum(sizes[sizes > (1 << 13)]))
