"""The autotuner's tables on the CPU (no GPU): the text format of
spdinv_tuning_save / spdinv_tuning_load, the rejection of malformed files,
and the application of a tuned batched schedule to the dispatch order the
host builds (a batch whose composition was tuned to one workgroup per
matrix gets one ticket per matrix)."""
import pytest

import paper_1002_4057_amd as spd


@pytest.fixture(autouse=True)
def _clean_tables():
    spd.tuning_clear()
    yield
    spd.tuning_clear()


def _counts(orders):
    c = [0] * 17
    for n in orders:
        c[1 if n <= 128 else -(-n // 128)] += 1
    return c


def test_round_trip_and_batched_entry_applies(tmp_path):
    orders = [200, 300, 90, 700]
    f = tmp_path / "tune.txt"
    f.write_text("spdinv-tuning 1\nfp64 32 1 12 4\nbatch 0 -1 4 " +
                 " ".join(map(str, _counts(orders))) + "\n")
    spd.tuning_load(str(f))
    plan = spd.batch_plan_export(orders, workers=512)
    assert len(plan["disp"]) == len(orders)          # one ticket per matrix
    other = spd.batch_plan_export(orders + [300], workers=512)   # another composition
    assert len(other["disp"]) > len(orders) + 1
    g = tmp_path / "again.txt"
    spd.tuning_save(str(g))
    assert g.read_text() == f.read_text()
    spd.tuning_clear()
    assert len(spd.batch_plan_export(orders, workers=512)["disp"]) > len(orders)


@pytest.mark.parametrize("text", [
    "not-a-tuning-file 1\n",
    "spdinv-tuning 2\n",
    "spdinv-tuning 1\nfp64 32 3 8 2\n",          # per_cu 3
    "spdinv-tuning 1\nfp64 32 1 8 3\n",          # three parts
    "spdinv-tuning 1\nbatch 0 -3 4 " + "0 " * 17 + "\n",
    "spdinv-tuning 1\nbatch 0 -1 4 1 2\n",       # counts cut short
    "spdinv-tuning 1\nsomething 1\n",
])
def test_malformed_files_are_rejected_and_add_nothing(tmp_path, text):
    f = tmp_path / "bad.txt"
    f.write_text(text)
    with pytest.raises(OSError):
        spd.tuning_load(str(f))
    g = tmp_path / "empty.txt"
    spd.tuning_save(str(g))
    assert g.read_text() == "spdinv-tuning 1\n"


def test_missing_file():
    with pytest.raises(OSError):
        spd.tuning_load("/nonexistent/dir/tune.txt")
