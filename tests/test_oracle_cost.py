"""The paper's cost formula reproduces the modelled column of tab:cost
(values stored in tests/golden/tab_cost.json, copied from that table)."""
import json
import os

from oracle.cost import cost, model_ratio

HERE = os.path.dirname(__file__)


def test_tab_cost_modelled_column():
    rows = json.load(open(os.path.join(HERE, "golden", "tab_cost.json")))["rows"]
    for r in rows:
        ratios = [1.0 if b is None else model_ratio(r["L"], b) for b in r["blocks"]]
        assert round(cost(r["n_eta"], ratios), 1) == r["modelled"], r


def test_dimension_ratio_g7():
    # the L2 operator of G7 (8^4 blocks, N_s N_c = 100) is about 500x smaller
    assert abs(model_ratio((128, 64, 64, 64), (8, 8, 8, 8)) - 491.52) < 1e-9
