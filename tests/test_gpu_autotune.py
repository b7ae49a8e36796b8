"""The autotuner on the GPU (spdinv_autotune, spdinv_autotune_batched through
the C-ABI): it times schedules on synthetic matrices and installs the
fastest as the library's choice; schedules change only the order of the
tasks, so results after tuning are the same bits as with the built-in
choice, and the tuned choice is one of the candidates."""
import pytest

import paper_1002_4057_amd as spd
from paper_1002_4057_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(autouse=True)
def _clean_tables():
    spd.tuning_clear()
    yield
    spd.tuning_clear()


def test_autotune_single_matrix_form():
    n = 3000
    a = inputs.wishart_shift(n, seed=21).to(DEV)
    before = spd.spd_inverse(a)
    tn = spd.autotune(n, reps=2)
    print("tuned:", tn, flush=True)
    assert tn["nb"] == 128 and tn["per_cu"] in (1, 2) and tn["chain"] in (6, 8, 12)
    assert tn["parts"] in (0, 2, 4) and 0 < tn["ms"] <= tn["ms_default"]
    assert 4 <= tn["candidates"] <= 8
    assert torch.equal(spd.spd_inverse(a), before)


def test_autotune_batched_form_and_tuning_file(tmp_path):
    orders = inputs.batch_orders(600, 16, 512, seed=22)
    mats = [m.to(DEV) for m in inputs.batched_wishart(orders, seed=22, shift=0.1)]
    before = spd.batched_spd_inverse(mats)
    tb = spd.autotune_batched(orders, "fp64", reps=2)
    print("tuned:", tb, flush=True)
    assert tb["batch_group"] in (-1, -2, 512) and tb["chain"] in (1, 4, 8)
    assert tb["candidates"] == 9 and 0 < tb["ms"] <= tb["ms_default"]
    after = spd.batched_spd_inverse(mats)
    assert all(torch.equal(x, y) for x, y in zip(before, after))
    f = tmp_path / "tune.txt"
    spd.tuning_save(str(f))
    spd.tuning_clear()
    spd.tuning_load(str(f))
    assert all(torch.equal(x, y) for x, y in zip(before, spd.batched_spd_inverse(mats)))
    t32 = spd.autotune_batched(orders, "fp32", reps=2)
    assert t32["batch_group"] in (-1, -2, 512) and t32["chain"] in (1, 4, 8)
    assert t32["candidates"] == 9
