"""The paper's qualitative findings, reproduced on the GPU path (reduced sizes
of bench.py --workload studies):
  Sec. 3.1 / Fig. 1: DGM is robust to the inner accuracy eps_in, DFGM is not;
  Sec. 6.3 / Fig. 5: outer iterations depend mildly on n, and the last primal
  iterate needs fewer than the averaged one."""
import numpy as np
import pytest

import bench
from paper_1504_05708_amd import duq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    duq.lib()


def test_inner_accuracy_sensitivity():
    print("[case] study: inner accuracy", flush=True)
    out = bench.study_inner_accuracy(seeds=range(501, 504), eps_ins=(1e-1, 1e-6), K=600, checkpoints=(200, 600))
    r = {(row["method"], row["eps_in"]): row for row in out["rows"]}
    # DGM: the same suboptimality at k = 200 whatever eps_in
    a, b = r[("DGM", 1e-1)]["subopt_rel"]["200"], r[("DGM", 1e-6)]["subopt_rel"]["200"]
    assert max(a, b) <= 1.5 * min(a, b)
    # DFGM: a coarse eps_in leaves it an order of magnitude less feasible
    assert r[("DFGM", 1e-1)]["feas"]["600"] >= 10.0 * r[("DFGM", 1e-6)]["feas"]["600"]


def test_outer_iterations_against_n():
    print("[case] study: outer iterations vs n", flush=True)
    out = bench.study_outer_vs_n(ns=(10, 100), per_n=5)
    for row in out["rows"]:
        for m in ("DGM", "DFGM"):
            assert row[f"{m}-LAST"]["ok"] == 5 and row[f"{m}-AVG"]["ok"] == 5
            assert row[f"{m}-LAST"]["mean_outer"] < row[f"{m}-AVG"]["mean_outer"]
    small, large = out["rows"][0], out["rows"][1]
    # tenfold n: the outer count grows by far less than tenfold
    assert large["DFGM-LAST"]["mean_outer"] <= 4.0 * small["DFGM-LAST"]["mean_outer"]
