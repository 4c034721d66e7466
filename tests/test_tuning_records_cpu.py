"""The tuning records shipped beside the library name configurations that
exist: every record's variant indexes lie within the library's compiled
configurations for its size and precision (one-pass records: whole-transform
configurations; two-pass records: the column and row configurations of the
split), so a change to the configuration list that drops an entry a record
points at fails here instead of on the device."""
import os

from paper_2604_00567_amd import binding

RECORDS = os.path.join(os.path.dirname(binding.LIB_PATH), "tuning_records.txt")
DTYPES = {0: "f16", 1: "f32", 2: "f16f32"}


def _records():
    with open(RECORDS) as fh:
        return [line.split() for line in fh if line.strip() and not line.startswith("#")]


def test_record_format():
    rows = _records()
    assert rows
    seen = set()
    for r in rows:
        assert len(r) == 8, r
        arch, cus, dtype, log2n, va, vb, two_pass, gbs = r
        assert arch.startswith("gfx") and int(cus) > 0 and int(dtype) in DTYPES
        assert 1 <= int(log2n) <= 20 and int(two_pass) in (0, 1) and float(gbs) > 0
        key = (arch, cus, dtype, log2n)
        assert key not in seen, key          # one record per size, precision and device
        seen.add(key)


def test_records_point_at_compiled_configurations():
    for arch, cus, dtype, log2n, va, vb, two_pass, gbs in _records():
        dt = DTYPES[int(dtype)]
        single, cols, rows = binding.fft_config_count(1 << int(log2n), dt)
        if int(two_pass):
            assert 0 <= int(va) < cols and 0 <= int(vb) < rows, (dt, log2n, va, vb)
        else:
            assert 0 <= int(va) < single and int(vb) == 0, (dt, log2n, va)
