"""Host logic without a GPU: the library's parameter planner (duq_plan_params,
Sec. 3.1 eq. choose_ein and Sec. 5) against the oracle's."""
import math

import pytest

from oracle import dfom
from oracle import plan as oplan
from paper_1504_05708_amd import duq


@pytest.mark.parametrize("method", [duq.DGM, duq.DFGM])
@pytest.mark.parametrize("eps,Ld,Rd,L_in,sigma,D_U", [(1e-2, 540.0, 3.0, 5.9, 0.27, 14.1),
                                                       (1e-4, 1.37e5, 40.0, 5.95, 0.178, 181.0),
                                                       (1e-3, 2.0, 0.5, 24000.0, 0.0, 90.5)])
def test_library_plan_matches_oracle(method, eps, Ld, Rd, L_in, sigma, D_U):
    got = duq.plan_params(method, eps, Ld, Rd, L_in, sigma, D_U)
    ref = oplan.plan(dfom.DGM if method == duq.DGM else dfom.DFGM, eps, Ld, Rd, L_in, sigma, D_U)
    assert math.isclose(got["eps_in"], ref.eps_in, rel_tol=1e-15)
    assert got["k_out"] == ref.k_out and got["k_in"] == ref.k_in and got["k_total"] == ref.k_total
    assert math.isclose(got["rho_star"], ref.rho_star, rel_tol=1e-15)


def test_library_plan_rejects_bad_input():
    for args in ((5, 1e-2, 1.0, 1.0), (duq.DGM, 0.0, 1.0, 1.0), (duq.DFGM, 1e-2, -1.0, 1.0),
                 (duq.DFGM, 1e-2, 1.0, 0.0), (duq.DGM, float("nan"), 1.0, 1.0)):
        with pytest.raises(duq.DuqError) as e:
            duq.plan_params(*args)
        assert e.value.code == duq.DUQ_EINVAL


def test_tuning_table_round_trip(tmp_path):
    # the tuning table is host data: records load, save back unchanged, and a
    # malformed file is refused
    src = tmp_path / "tune.txt"
    src.write_text("0 0 4 2\n1 1 2 3\n")
    duq.tune_load(str(src))
    out = tmp_path / "out.txt"
    duq.tune_save(str(out))
    lines = set(out.read_text().split("\n")) - {""}
    assert {"0 0 4 2", "1 1 2 3"} <= lines
    bad = tmp_path / "bad.txt"
    bad.write_text("0 0 4 9\n")
    with pytest.raises(duq.DuqError) as e:
        duq.tune_load(str(bad))
    assert e.value.code == duq.DUQ_EINVAL
