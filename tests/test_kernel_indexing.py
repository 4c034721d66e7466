"""CPU simulation of the FFT kernel's per-lane index arithmetic (no GPU).

Replays, lane by lane, the addressing of fft_unit_kernel for every compiled
configuration: global loads/stores, the padded LDS exchange between register
passes, and the twiddle entries, with FP64 butterflies.  It checks that every
access stays inside its buffer, that each output is written exactly once, that
each LDS read sees a value written in the same exchange, and that the result is
the DFT.  This guards the index math before it runs on the GPU.
"""
import os
import re

import numpy as np
import pytest

from paper_2604_00567_amd import binding

CONFIGS = os.path.join(os.path.dirname(os.path.dirname(__file__)),
                       "paper_2604_00567_amd", "csrc", "configs.inc")
MODES = {"MODE_SMALL": 0, "MODE_COLS": 1, "MODE_ROWS": 2}


def load_configs(with_upl=False):
    out = []
    for line in open(CONFIGS):
        # CFG(10 fields), CFGU(..., UPL), CFGE(..., UPL, ENC); the path
        # encoding changes no index
        m = re.match(r"\s*CFG(U|E)?\((\w+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),"
                     r"\s*(\d+),\s*(\d+),\s*(\d+)(?:,\s*(\d+))?(?:,\s*(ENC_\w+))?\)", line)
        if m:
            mode = MODES[m.group(2)]
            upl = int(m.group(12)) if m.group(1) else 1
            assert (m.group(1) == "E") == (m.group(13) is not None)
            # the pipelined flag changes which workgroup takes a block, not a
            # block's index math (blocks b, b + grid, ... cover every block once)
            cfg = (mode,) + tuple(int(m.group(i)) for i in range(3, 11))
            out.append(cfg + (upl,) if with_upl else cfg)
    return out


class PassPlan:
    def __init__(self, log_nu, lrs, lane=0):
        self.log_nu = log_nu
        self.lrs = [x for x in lrs if x]
        self.np = len(self.lrs)
        self.lane = lane

    def lr(self, p):
        return self.lrs[p]

    def log_l0(self, p):
        return sum(self.lrs[:p])

    def log_m(self, p):
        return self.log_nu - self.log_l0(p) - self.lr(p)

    def pad(self, p):
        if self.lane and p + 2 == self.np:
            return 2
        return (1 << self.log_m(p + 1)) if (p + 1 < self.np and self.log_m(p + 1) < 5) else 0

    def padded(self, p):
        return (1 << self.log_nu) + ((1 << self.log_nu) >> self.log_m(p)) * self.pad(p)

    def region(self):
        r = 1 << self.log_nu
        for p in range(self.np - 1):
            r = max(r, self.padded(p))
        return r | 1

    def half_region(self):
        return max(self.padded(p) // 2 for p in range(self.np - 1))


LDS_BYTES = 160 * 1024


def exchange_rounds(pp, mode, upw, log_e, esize):
    """Two rounds (half of the exchange's rows each) for a lone whole-transform
    unit whose exchange does not fit, or whose CU holds fewer than the 16
    waves that lanes of 256 bytes or more leave registers for and would hold
    more workgroups with the exchange halved, when each later pass has two or
    more groups per lane."""
    if not (mode == 0 and upw == 1 and pp.np > 1):
        return 1
    if any(pp.lr(p) >= log_e for p in range(1, pp.np)):
        return 1
    one, two = pp.region() * esize, pp.half_region() * esize
    if one > LDS_BYTES:
        return 2
    if (esize << log_e) < 256:
        return 1
    waves = max(1, (1 << (pp.log_nu - log_e)) // 64)
    wg1, wg2 = LDS_BYTES // one, LDS_BYTES // two
    return 2 if (wg1 * waves < 16 and wg2 > wg1) else 1


def lds_elems(pp, mode, upw, log_e, esize):
    if exchange_rounds(pp, mode, upw, log_e, esize) == 2:
        return pp.half_region()
    return upw * pp.region()


def level_twiddle(idx):
    """Entry idx of the level-ordered table: L/2 + j -> W_L^j."""
    L = 1
    while L <= idx:
        L <<= 1
    j = idx - L // 2
    return np.exp(-2j * np.pi * j / L), L, j


def bfly(a, b, w):
    return a + w * b, a - w * b


def swap_halves(x, y, d):
    """Model of v_permlane{32,16}_swap on one wave (64 lanes): lanes whose bit
    d is clear receive into y the x of lane l + d; lanes with the bit set
    receive into x the y of lane l - d."""
    x2, y2 = x.copy(), y.copy()
    for l in range(64):
        if l & d:
            x2[l] = y[l - d]
        else:
            y2[l] = x[l + d]
    return x2, y2


def lane_tail_model(v, NU, EL, NT, tcap):
    """The two cross-lane stages of fft_device.hpp's lane_tail, per wave."""
    for w0 in range(0, NT, 64):
        lanes = np.arange(64)
        q, r, u = lanes & 15, (lanes >> 4) & 1, lanes >> 5
        for stage, d in ((1, 32), (2, 16)):
            for k in range(EL // 2):
                x, y = v[w0:w0 + 64, 2 * k].copy(), v[w0:w0 + 64, 2 * k + 1].copy()
                x, y = swap_halves(x, y, d)
                for l in range(64):
                    if stage == 1:
                        idx = NU // 4 + q[l] + 16 * (2 * k + u[l])
                        L_expect = NU // 2
                    else:
                        idx = NU // 2 + q[l] + 16 * (2 * k + u[l]) + (NU // 4) * r[l]
                        L_expect = NU
                    assert 0 < idx < tcap
                    w, L, j = level_twiddle(idx)
                    assert L == L_expect
                    x[l], y[l] = bfly(x[l], y[l], w)
                v[w0:w0 + 64, 2 * k], v[w0:w0 + 64, 2 * k + 1] = x, y


def simulate(cfg, n, batch, x=None, esize=4):
    mode, log_nu, log_e, upw, lr0, lr1, lr2, stg, lane = cfg
    pp = PassPlan(log_nu, (lr0, lr1, lr2), lane)
    NU, EL = 1 << log_nu, 1 << log_e
    G = NU // EL
    NT = upw * G
    RS = pp.region()
    XR = exchange_rounds(pp, mode, upw, log_e, esize)
    LDS = lds_elems(pp, mode, upw, log_e, esize)
    assert LDS * esize <= LDS_BYTES, "configuration does not fit"
    log_m = (n.bit_length() - 1) - log_nu
    units = batch if mode == 0 else batch << log_m
    if x is None:
        rng = np.random.default_rng(cfg[1] * 7 + cfg[3])
        x = rng.standard_normal(batch * n) + 1j * rng.standard_normal(batch * n)
    out = np.full(batch * n, np.nan + 0j)
    written = np.zeros(batch * n, int)
    tcap = max(n, 4096)
    grid = (units + upw - 1) // upw
    for blk in range(grid):
        lds = np.full(max(LDS, upw * RS), np.nan + 0j)
        lds_gen = np.full(max(LDS, upw * RS), -1)
        pre = None                                 # next pass's values (two-round exchange)
        v = np.zeros((NT, EL), complex)
        for p in range(pp.np):
            LR = pp.lr(p)
            R = 1 << LR
            L0 = 1 << pp.log_l0(p)
            LOGM = pp.log_m(p)
            M = 1 << LOGM
            GPL = EL // R
            unit_fast = mode == 1 or (mode == 2 and p == pp.np - 1)
            newv = np.zeros_like(v)
            geos = []
            for tid in range(NT):
                ul = tid % upw if unit_fast else tid // G
                g0 = tid // upw if unit_fast else tid % G
                g = (((g0 & 15) << 2) | (g0 >> 4)) if (lane and p == pp.np - 1) else g0
                unit = blk * upw + ul
                active = unit < units
                reg = ul * RS
                if mode == 0:
                    base_in = base_out = unit << log_nu
                    in_s = out_s = 1
                    q0, log_lb = 0, 0
                elif mode == 1:
                    b, r0 = unit >> log_m, unit & ((1 << log_m) - 1)
                    base_in = base_out = (b << (log_m + log_nu)) + r0
                    in_s = out_s = 1 << log_m
                    q0, log_lb = 0, 0
                else:
                    b, q0 = unit >> log_m, unit & ((1 << log_m) - 1)
                    log_lb = log_m
                    base_in = (b << (log_m + log_nu)) + (q0 << log_nu)
                    base_out = (b << (log_m + log_nu)) + q0
                    in_s, out_s = 1, 1 << log_m
                vv = v[tid].copy() if p > 0 else np.zeros(EL, complex)
                # gather
                for u in range(GPL):
                    gam = g + G * u
                    if p == 0 and stg:
                        # staged: the block sits in LDS in natural order
                        # (whole transforms, or consecutive workspace rows)
                        assert mode in (0, 2) and EL * 4 >= 16
                        assert base_in == unit << log_nu
                        r = gam
                        for i in range(R):
                            idx = r + M * i
                            a = ul * NU + idx
                            assert a < upw * NU <= upw * RS
                            if active:
                                vv[u * R + i] = x[base_in + idx]
                    elif p == 0:
                        r = gam
                        for i in range(R):
                            idx = r + M * i
                            assert idx < NU
                            if active:
                                a = base_in + idx * in_s
                                assert 0 <= a < batch * n
                                vv[u * R + i] = x[a]
                    elif XR == 2:
                        vv[u * R:(u + 1) * R] = pre[tid][u * R:(u + 1) * R]
                    else:
                        padp = pp.pad(p - 1)
                        r, q = gam & (M - 1), gam >> LOGM
                        basep = r + ((NU // L0) + padp) * q
                        for i in range(R):
                            a = reg + basep + M * i
                            assert reg <= a < reg + RS and basep + M * i < RS
                            assert lds_gen[a] == p - 1, "LDS read of a slot not written"
                            vv[u * R + i] = lds[a]
                # stages
                for u in range(GPL):
                    gam = g + G * u
                    q = gam >> LOGM
                    if p == 0 and mode != 2:
                        tw_idx = [c for c in range(R)]
                    else:
                        qg = q0 + (q << log_lb)
                        lg0 = L0 << log_lb
                        tw_idx = [qg + lg0 * c for c in range(R)]
                    grp = vv[u * R:(u + 1) * R].copy()
                    for t in range(1, LR + 1):
                        H = R >> t
                        nv = np.zeros(R, complex)
                        for e in range(1 << (t - 1)):
                            c = (1 << (t - 1)) + e
                            assert 0 < tw_idx[c] < tcap
                            w, L, j = level_twiddle(tw_idx[c])
                            # the twiddle must be W_{L}^{j} with L the global span
                            assert L == (L0 << log_lb) * (1 << t) and j < L // 2
                            for i in range(H):
                                A, B = bfly(grp[i + 2 * H * e], grp[i + H + 2 * H * e], w)
                                nv[i + H * e] = A
                                nv[i + H * e + R // 2] = B
                        grp = nv
                    vv[u * R:(u + 1) * R] = grp
                newv[tid] = vv
                geos.append((ul, g, active, reg, base_out, out_s))
            if lane and p == pp.np - 1:
                assert G == 64 and GPL == 1 and M == 4 and L0 == 16 and mode == 0
                lane_tail_model(newv, NU, EL, NT, tcap)
            if XR == 2 and p + 1 < pp.np:
                # two rounds of half the rows: writes of elements e in half h,
                # then reads of the next pass's groups u1 in half h
                pad = pp.pad(p)
                NR = L0 * R
                R1, LOGM1 = 1 << pp.lr(p + 1), pp.log_m(p + 1)
                M1, GPL1 = 1 << LOGM1, EL // (1 << pp.lr(p + 1))
                assert GPL1 >= 2 and upw == 1 and not lane and not stg
                pre = np.full((NT, EL), np.nan + 0j)
                for h in range(2):
                    gen = 100 + 2 * p + h
                    for tid in range(NT):
                        g = tid % G
                        for u in range(GPL):
                            gam = g + G * u
                            r, q = gam & (M - 1), gam >> LOGM
                            for e in range(h * (R // 2), (h + 1) * (R // 2)):
                                a = r + (M + pad) * (q + L0 * e - h * (NR // 2))
                                assert 0 <= a < LDS, "round write outside the half region"
                                assert lds_gen[a] != gen, "two writes to one LDS slot in a round"
                                lds[a] = newv[tid][u * R + e]
                                lds_gen[a] = gen
                    for tid in range(NT):
                        g = tid % G
                        for u1 in range(h * (GPL1 // 2), (h + 1) * (GPL1 // 2)):
                            gam1 = g + G * u1
                            r1, q1 = gam1 & (M1 - 1), gam1 >> LOGM1
                            basep = r1 + (M + pad) * (q1 - h * (NR // 2))
                            for i in range(R1):
                                a = basep + M1 * i
                                assert 0 <= a < LDS
                                assert lds_gen[a] == gen, "round read of a slot not written in it"
                                pre[tid][u1 * R1 + i] = lds[a]
                assert not np.any(np.isnan(pre))
                v = newv
                continue
            # every lane has gathered before any lane scatters (the kernel's barrier)
            for tid in range(NT):
                ul, g, active, reg, base_out, out_s = geos[tid]
                vv = newv[tid]
                if lane and p == pp.np - 1:
                    g0 = tid % G
                    q, r, u = g0 & 15, (g0 >> 4) & 1, g0 >> 5
                    for k in range(EL // 2):
                        jb = q + 16 * (2 * k + u) + (NU // 4) * r
                        for idx, val in ((jb, vv[2 * k]), (jb + NU // 2, vv[2 * k + 1])):
                            assert idx < NU
                            if active:
                                a = base_out + idx
                                assert 0 <= a < batch * n
                                out[a] = val
                                written[a] += 1
                    continue
                if p + 1 < pp.np:
                    pad = pp.pad(p)
                    for u in range(GPL):
                        gam = g + G * u
                        r, q = gam & (M - 1), gam >> LOGM
                        for e in range(R):
                            a = reg + r + (M + pad) * (q + L0 * e)
                            assert reg <= a < reg + RS
                            assert lds_gen[a] < p, "two writes to one LDS slot"
                            lds[a] = vv[u * R + e]
                            lds_gen[a] = p
                else:
                    for u in range(GPL):
                        q = g + G * u
                        for e in range(R):
                            idx = q + L0 * e
                            assert idx < NU
                            if stg:
                                assert ul * NU + idx < upw * NU <= upw * RS
                            if active:
                                a = base_out + idx * out_s
                                assert 0 <= a < batch * n
                                out[a] = vv[u * R + e]
                                written[a] += 1
            v = newv
    return x, out, written, units


@pytest.mark.parametrize("cfg", [c for c in load_configs() if c[0] == 0])
def test_small_configs_index_math(cfg):
    n = 1 << cfg[1]
    batch = cfg[3] + 1                            # ragged tail: one extra unit
    x, out, written, _ = simulate(cfg, n, batch)
    assert np.all(written == 1)
    ref = np.fft.fft(x.reshape(batch, n), axis=1).ravel()
    assert np.max(np.abs(out - ref)) < 1e-9 * n


def test_configs_parsed():
    cfgs = load_configs()
    text = open(CONFIGS).read()
    assert len(cfgs) == text.count("\nCFG(") + text.count("\nCFGU(") + text.count("\nCFGE(") and len(cfgs) > 40


def lane_units(tid, G, upw, upl):
    """Units and group position of lane tid in a whole-transform workgroup
    with upl units per lane (the kernel's mapping)."""
    return [(tid // G) * upl + k for k in range(upl)], tid % G


@pytest.mark.parametrize("cfg", [c for c in load_configs(with_upl=True) if c[-1] > 1])
def test_units_per_lane_mapping(cfg):
    # (lane, k) -> (unit, group position) covers the workgroup's units and
    # positions exactly once, as the one-unit-per-lane mapping of the same
    # configuration does; every other index is that configuration's
    mode, log_nu, log_e, upw = cfg[:4]
    upl = cfg[-1]
    assert mode == 0 and upw % upl == 0 and cfg[8] == 0
    G = 1 << (log_nu - log_e)
    nt = (upw // upl) * G
    seen = set()
    for tid in range(nt):
        units, g = lane_units(tid, G, upw, upl)
        for ul in units:
            assert 0 <= ul < upw and 0 <= g < G
            seen.add((ul, g))
    assert seen == {(ul, g) for ul in range(upw) for g in range(G)}
    # per unit, the lanes' work is the one-unit-per-lane configuration's
    n = 1 << log_nu
    x, out, written, _ = simulate(cfg[:9], n, upw + 1)
    assert np.all(written == 1)
    ref = np.fft.fft(x.reshape(upw + 1, n), axis=1).ravel()
    assert np.max(np.abs(out - ref)) < 1e-9 * n


def test_persistent_blocks_cover_once():
    for nblk in (1, 7, 256, 1000):
        for grid in (1, 3, 256, 2048):
            g = min(grid, nblk)
            seen = [b for w in range(g) for b in range(w, nblk, g)]
            assert sorted(seen) == list(range(nblk))


@pytest.mark.parametrize("m1,m2,rows_staged", [(6, 6, 0), (7, 6, 0), (7, 7, 0), (8, 6, 0), (7, 7, 1),
                                                (8, 7, 1), (8, 8, 1)])
def test_two_pass_index_math(m1, m2, rows_staged):
    cfgs = load_configs()
    cols = next(c for c in cfgs if c[0] == 1 and c[1] == m1)
    rows = next(c for c in cfgs if c[0] == 2 and c[1] == m2 and c[7] == rows_staged)
    assert cols[-1] == 0 and rows[-1] == 0
    n = 1 << (m1 + m2)
    batch = 2
    x, ws, w1, _ = simulate(cols, n, batch)
    assert np.all(w1 == 1)
    _, out, w2, _ = simulate(rows, n, batch, x=ws)
    assert np.all(w2 == 1)
    ref = np.fft.fft(x.reshape(batch, n), axis=1).ravel()
    assert np.max(np.abs(out - ref)) < 1e-9 * n


BATCH_SRC = os.path.join(os.path.dirname(os.path.dirname(__file__)),
                         "paper_2604_00567_amd", "csrc", "fft_batch.hpp")


def load_batch_configs():
    """The uneven-batch kernel's configurations, as (name, config tuple)."""
    out = {}
    for line in open(BATCH_SRC):
        m = re.match(r"\s*case (HB_\w+): batch_unit<E, (\d+), (\d+), (\d+), (\w+), (\d+), (\d+), "
                     r"(\d+)>", line)
        if m:
            lognu, loge, upw = int(m.group(2)), int(m.group(3)), int(m.group(4))
            lrs = tuple(int(m.group(i)) for i in (6, 7, 8))
            out[m.group(1)] = (MODES[m.group(5)], lognu, loge, upw) + lrs + (0, 0)
    return out


def test_batch_configs_parsed():
    cfgs = load_batch_configs()
    assert len(cfgs) == 25
    for name, c in cfgs.items():
        assert c[3] << (c[1] - c[2]) == 512, name       # every configuration uses 512 threads
        assert sum(c[4:7]) == c[1], name


@pytest.mark.parametrize("name", [n for n, c in load_batch_configs().items() if c[0] == 0])
def test_batch_small_configs_index_math(name):
    cfg = load_batch_configs()[name]
    n = 1 << cfg[1]
    batch = cfg[3] + 1
    x, out, written, _ = simulate(cfg, n, batch)
    assert np.all(written == 1)
    ref = np.fft.fft(x.reshape(batch, n), axis=1).ravel()
    assert np.max(np.abs(out - ref)) < 1e-9 * n


@pytest.mark.parametrize("cols,rows", [("HB_COLS256", "HB_ROWS128"),
                                       ("HB_COLS256", "HB_ROWS256"), ("HB_COLS512", "HB_ROWS256"),
                                       ("HB_COLS512", "HB_ROWS512")])
def test_batch_two_pass_index_math(cols, rows):
    cfgs = load_batch_configs()
    c, r = cfgs[cols], cfgs[rows]
    n = 1 << (c[1] + r[1])
    batch = 1
    x, ws, w1, _ = simulate(c, n, batch)
    assert np.all(w1 == 1)
    _, out, w2, _ = simulate(r, n, batch, x=ws)
    assert np.all(w2 == 1)
    ref = np.fft.fft(x.reshape(batch, n), axis=1).ravel()
    assert np.max(np.abs(out - ref)) < 1e-9 * n


@pytest.mark.parametrize("cfg", [c for c in load_configs() if c[0] in (1, 2)])
def test_every_column_and_row_config_index_math(cfg):
    """Each column (row) configuration paired with a row (column) configuration
    of the same size: the pair computes the DFT, every workspace and output
    element written once."""
    cfgs = load_configs()
    mode = cfg[0]
    # the smallest configuration of the other kind keeps the simulated size down
    other = min((c for c in cfgs if c[0] == 3 - mode and c[7] == 0), key=lambda c: (c[1], c[3]))
    cols, rows = (cfg, other) if mode == 1 else (other, cfg)
    n = 1 << (cols[1] + rows[1])
    x, ws, w1, _ = simulate(cols, n, 1)
    assert np.all(w1 == 1)
    _, out, w2, _ = simulate(rows, n, 1, x=ws)
    assert np.all(w2 == 1)
    ref = np.fft.fft(x.reshape(1, n), axis=1).ravel()
    assert np.max(np.abs(out - ref)) < 1e-9 * n


def load_full_configs():
    """(mode, log_nu, log_e, upw, lr0, lr1, lr2, stg, lane, pipe, upl, enc) of
    every entry, in registry order."""
    out = []
    for line in open(CONFIGS):
        m = re.match(r"\s*CFG(U|E)?\((\w+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),"
                     r"\s*(\d+),\s*(\d+),\s*(\d+)(?:,\s*(\d+))?(?:,\s*(ENC_\w+))?\)", line)
        if m:
            upl = int(m.group(12)) if m.group(1) else 1
            enc = m.group(13) or "ENC_TABLE"
            out.append((MODES[m.group(2)],) + tuple(int(m.group(i)) for i in range(3, 12)) + (upl, enc))
    return out


def lds_twiddle_last_pass(pp, log_nu, log_e, mode, lane, pipe=3):
    """Last pass a PIPE = 3 workgroup serves from LDS (from pass 1 on): the
    middle pass of a three-pass whole transform unless its column is
    wave-uniform (scalar loads), every later pass of a column unit; PIPE = 4:
    every pass after the first of a whole transform; PIPE = 5 as PIPE = 3
    (its prefetch serves the other passes); 0: none."""
    if lane or pipe not in (3, 4, 5):
        return 0
    if mode == 1 or (mode == 0 and pipe == 4):
        return pp.np - 1 if pp.np >= 2 else 0
    if mode != 0 or pp.np != 3:
        return 0
    G = (1 << log_nu) >> log_e
    if pp.log_m(1) >= 6 and G % 64 == 0:
        return 0
    return 1


def lds_twiddle_entries(pp, log_nu, log_e, mode, lane, pipe=3):
    """Table entries [L0 of pass 1, L0 R of the last served pass) in the copy."""
    last = lds_twiddle_last_pass(pp, log_nu, log_e, mode, lane, pipe)
    if last == 0:
        return 0
    return (1 << (pp.log_l0(last) + pp.lr(last))) - (1 << pp.log_l0(1))


def lds_row_twiddle_entries(c):
    """Row units, PIPE = 3: entry (c, unit) of the first pass per workgroup."""
    mode, log_nu, log_e, upw, lr0, lr1, lr2, stg, lane, pipe, upl, enc = c
    return ((1 << lr0) - 1) * upw if (mode == 2 and pipe == 3) else 0


def lds_bytes(c, esize, twsize):
    mode, log_nu, log_e, upw, lr0, lr1, lr2, stg, lane, pipe, upl, enc = c
    pp = PassPlan(log_nu, (lr0, lr1, lr2), lane)
    ex = lds_elems(pp, mode, upw, log_e, esize) * esize
    te = lds_twiddle_entries(pp, log_nu, log_e, mode, lane, pipe) + lds_row_twiddle_entries(c)
    return ex if te == 0 else (ex + 15) // 16 * 16 + te * twsize


def compiled(c, dtype):
    """The registry's rule (cfg_fits) for an entry and a plan precision."""
    mode, log_nu, log_e, upw, lr0, lr1, lr2, stg, lane, pipe, upl, enc = c
    esize, twsize = (4, 8) if dtype == "f16" else (8, 16)
    if enc == "ENC_RADIX4":
        # the radix-4 form: stored as computed, whole transforms, no lane tail,
        # no second register set or prefetch, passes on radix-4 stage boundaries;
        # its table entries are 32 / 64 bytes
        if dtype == "f16f32" or mode != 0 or lane or pipe in (1, 2, 5):
            return False
        if lr0 % 2 != log_nu % 2 or lr1 % 2 or lr2 % 2:
            return False
        twsize *= 4
    if dtype == "f16f32" and ((stg and lane) or pipe == 1):
        return False
    if enc not in ("ENC_TABLE", "ENC_RADIX4") and (dtype != "f16" or pipe == 1 or lane):
        return False
    pp = PassPlan(log_nu, (lr0, lr1, lr2), lane)
    if stg and exchange_rounds(pp, mode, upw, log_e, esize) == 2:
        return False
    if pipe in (3, 4, 5) and lds_twiddle_entries(pp, log_nu, log_e, mode, lane, pipe) == 0 \
            and lds_row_twiddle_entries(c) == 0:
        return False
    return lds_bytes(c, esize, twsize) <= LDS_BYTES


def two_pass_split(m, dtype):
    """(column, row) log2 NU of the two-pass schedule for N = 2^m, as the
    library splits it (columns take the larger half)."""
    c = (m + 1) // 2
    return c, m - c


@pytest.mark.parametrize("dtype", ["f16", "f32", "f16f32"])
def test_compiled_configurations_match_the_model(dtype):
    """The library's count of configurations per size (whole transforms,
    columns, rows) is the count of entries the LDS model and the precision
    rules admit."""
    full = load_full_configs()
    for m in range(1, 21):
        single, cols, rows = binding.fft_config_count(1 << m, dtype)
        want = sum(1 for c in full if c[0] == 0 and c[1] == m and c[11] != "ENC_RADIX4" and compiled(c, dtype))
        assert single == want, (m, dtype)
        want4 = sum(1 for c in full if c[0] == 0 and c[1] == m and c[11] == "ENC_RADIX4" and compiled(c, dtype))
        assert binding.fft_config_count_radix4(1 << m, dtype) == want4, (m, dtype)
        lc, lr = two_pass_split(m, dtype)
        assert cols == sum(1 for c in full if c[0] == 1 and c[1] == lc and compiled(c, dtype)), (m, dtype)
        assert rows == sum(1 for c in full if c[0] == 2 and c[1] == lr and compiled(c, dtype)), (m, dtype)


@pytest.mark.parametrize("cfg", [c for c in load_full_configs() if c[9] == 3 and c[0] == 2])
@pytest.mark.parametrize("esize,twsize", [(4, 8), (8, 16)])
def test_lds_row_twiddle_copy(cfg, esize, twsize):
    """Row units, PIPE = 3: the copy loop writes slot (c - 1) UPW + unit once
    for every first-pass entry c of every unit, after the exchange area, and
    each lane of unit ul reads slot (c - 1) UPW + ul, the entry q0 + c 2^log_m
    of its own row."""
    mode, log_nu, log_e, upw, lr0, lr1, lr2, stg, lane, pipe, upl, enc = cfg
    pp = PassPlan(log_nu, (lr0, lr1, lr2), lane)
    if lds_bytes(cfg, esize, twsize) > LDS_BYTES:
        pytest.skip("not compiled for this element size")
    te = lds_row_twiddle_entries(cfg)
    R0 = 1 << lr0
    G = (1 << log_nu) >> log_e
    nt = upw * G
    for log_m in (6, 9):
        ublk = 3 * upw
        slots = {}
        for t in range(nt):
            for i in range(t, te, nt):
                c, ul = 1 + i // upw, i % upw
                q0 = (ublk + ul) & ((1 << log_m) - 1)
                assert i not in slots
                slots[i] = q0 + (c << log_m)
        assert sorted(slots) == list(range(te))
        for t in range(nt):
            ul = t // G
            q0 = (ublk + ul) & ((1 << log_m) - 1)
            for c in range(1, R0):
                assert slots[(c - 1) * upw + ul] == q0 + (c << log_m)
    ex = lds_elems(pp, mode, upw, log_e, esize) * esize
    assert (ex + 15) // 16 * 16 + te * twsize <= LDS_BYTES


@pytest.mark.parametrize("cfg", [c for c in load_full_configs() if c[9] in (3, 4, 5) and c[0] != 2])
@pytest.mark.parametrize("esize,twsize", [(4, 8), (8, 16)])
def test_lds_twiddle_copy(cfg, esize, twsize):
    """PIPE = 3, 4 and 5: the copy of the served passes' entries fills whole 16-byte
    chunks from a 16-byte aligned table offset, every chunk exactly once,
    after the exchange area; every lane's read in each served pass lands on
    the entry the table path reads (q + L0 c), inside the copy."""
    mode, log_nu, log_e, upw, lr0, lr1, lr2, stg, lane, pipe, upl, enc = cfg
    if enc == "ENC_RADIX4":
        twsize *= 4                               # radix-4 entries: 32 / 64 bytes
    pp = PassPlan(log_nu, (lr0, lr1, lr2), lane)
    te = lds_twiddle_entries(pp, log_nu, log_e, mode, lane, pipe)
    last = lds_twiddle_last_pass(pp, log_nu, log_e, mode, lane, pipe)
    assert mode in (0, 1) and te > 0, "a PIPE = 3, 4 or 5 entry needs a pass to serve"
    if lds_bytes(cfg, esize, twsize) > LDS_BYTES:
        pytest.skip("not compiled for this element size")
    ex = lds_elems(pp, mode, upw, log_e, esize) * esize
    off = (ex + 15) // 16 * 16
    L01 = 1 << pp.log_l0(1)
    assert (te * twsize) % 16 == 0 and (L01 * twsize) % 16 == 0 and off >= ex
    assert off + te * twsize <= LDS_BYTES
    G = (1 << log_nu) >> log_e
    nt = (upw // upl) * G
    chunks = te * twsize // 16
    seen = sorted(i for t in range(nt) for i in range(t, chunks, nt))
    assert seen == list(range(chunks))
    for p in range(1, last + 1):
        L0 = 1 << pp.log_l0(p)
        R = 1 << pp.lr(p)
        LOGM = pp.log_m(p)
        GPL = (1 << log_e) // R
        for t in range(nt):
            g = t // upw if mode == 1 else t % G      # column units: unit-fast lanes
            for u in range(GPL):
                q = (g + G * u) >> LOGM
                assert 0 <= q < L0
                for c in range(1, R):
                    idx = q + L0 * c - L01
                    assert 0 <= idx < te and L01 + idx == q + L0 * c


@pytest.mark.parametrize("cfg", [c for c in load_full_configs() if c[11] == "ENC_RADIX4"])
def test_radix4_entry_indices(cfg):
    """Radix-4 form: in pass P (span L0 before it, radix R) a lane's group in
    column q reads entries q + L0 c.  The stages of the pass read c = S + e
    (S columns done before the stage, e < S), which is entry L/4 + j of the
    radix-4 table for the stage's span L = 4 L0 S and column j = q + L0 e; the
    span-2 stage of an odd log2 N (first pass) reads entry 0.  Every index read
    lies below L0 R / 2 <= N/2, inside the table (N_cap entries), and the
    stages cover every (span, column) of the canonical radix-4 order once."""
    mode, log_nu, log_e, upw, lr0, lr1, lr2, stg, lane, pipe, upl, enc = cfg
    assert mode == 0 and lane == 0 and pipe not in (1, 2, 5)
    pp = PassPlan(log_nu, (lr0, lr1, lr2), lane)
    n = 1 << log_nu
    odd = log_nu % 2
    assert pp.lr(0) % 2 == odd and all(pp.lr(p) % 2 == 0 for p in range(1, pp.np))
    seen = set()
    for p in range(pp.np):
        L0, R = 1 << pp.log_l0(p), 1 << pp.lr(p)
        for q in range(L0):
            S = 1
            if p == 0 and odd:
                assert q == 0
                seen.add((2, 0))
                S = 2
            while S < R:
                for e in range(S):
                    c = S + e
                    assert (1 if not (p == 0 and odd) else 2) <= c < R // 2 or (R == 4 and c == 1)
                    idx = q + L0 * c
                    span, j = 4 * L0 * S, q + L0 * e
                    assert idx == span // 4 + j and j < span // 4
                    assert idx < max(L0 * R // 2, 2) <= max(n // 2, 2)
                    seen.add((span, j))
                S *= 4
    # the canonical radix-4 order: span 2 first when log2 N is odd, then every
    # radix-4 span up to N, each with its L/4 columns
    want = {(2, 0)} if odd else set()
    span = 8 if odd else 4
    while span <= n:
        want |= {(span, j) for j in range(span // 4)}
        span *= 4
    assert seen == want
