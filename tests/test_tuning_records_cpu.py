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


def test_record_file_reader_skips_comments_and_bad_lines(tmp_path):
    """A record file may hold comments, blank lines and malformed or
    out-of-range lines: each is skipped on its own and the records after it
    still apply.  Without a GPU the device tag reads 'unknown 0', so records
    carrying that tag are the ones a CPU process takes."""
    import subprocess
    import sys
    f = tmp_path / "records.txt"
    f.write_text("# a comment line\n"
                 "\n"
                 "unknown 0 0 10 not-a-number 0 0 1.0\n"
                 "unknown 0 7 11 0 0 0 1.0\n"          # unknown dtype
                 "unknown 0 0 12 0 0 2 1.0\n"          # two_pass must be 0 or 1
                 "   # indented comment\n"
                 "unknown 0 0 10 1 0 0 100.0\n"
                 "unknown 0 1 13 2 0 0 100.0\n"
                 "gfx000 1 1 14 3 0 0 100.0\n")        # another device
    code = ("from paper_2604_00567_amd import binding as b; "
            "print(b.fft_tuned_choice(1024, 'f16'), b.fft_tuned_choice(8192, 'f32'), "
            "b.fft_tuned_choice(2048, 'f16'), b.fft_tuned_choice(4096, 'f16'), b.fft_tuned_choice(16384, 'f32'))")
    env = dict(os.environ, DSFFT_TUNE_FILE=str(f), HIP_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env["PYTHONPATH"] = root + os.pathsep + env.get("PYTHONPATH", "")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split("\n")[0] == "(1, 0, False) (2, 0, False) None None None"
