"""Memory-constrained partial renaming on the GPU (spd_inverse with
opts.rename_tiles through the C-ABI): the renamed rows are read from their
copies and the others in place, with the same products in the same order per
tile, so every budget gives the bits of full renaming; the workspace shrinks
with the budget."""
import pytest

import paper_1002_4057_amd as spd
from paper_1002_4057_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.mark.parametrize("n", [700, 2000, 4097])
def test_budgets_give_the_bits_of_full_renaming(n):
    t = -(-n // 128)
    T = t * (t + 1) // 2
    a = inputs.wishart_shift(n, seed=50 + n).to(DEV)
    ref = spd.spd_inverse(a)
    full_ws = spd.workspace_bytes(n)
    for k in (1, T // 3, T, 3 * T // 2):
        x, rep = spd.spd_inverse(a, rename_tiles=k, return_report=True)
        print(f"n={n} budget={k}: critical path {rep['critical_path']}", flush=True)
        assert torch.equal(x, ref), k
        assert spd.workspace_bytes(n, rename_tiles=k) <= full_ws - (2 * T - k) * 128 * 128 * 8


def test_partial_renaming_in_place_ablation_bits():
    n = 1500
    a = inputs.wishart_shift(n, seed=7).to(DEV)
    # the same products per tile as the in-place plan of the same loop order
    for opts in (dict(rename_tiles=20, chain=1), dict(rename_tiles=40, pipelined=0),
                 dict(rename_tiles=30, loop_order=1), dict(rename_tiles=50, trtri_first=1)):
        ref = spd.spd_inverse(a, renamed=0, loop_order=opts.get("loop_order", 0))
        assert torch.equal(spd.spd_inverse(a, **opts), ref), opts
