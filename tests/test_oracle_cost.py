"""Pins for the cost model (Section 6.2) and Eq. 7 against the numbers the
paper prints in Section 6.3 and Table 1 (fixture: tests/golden/cost_model.json)."""
import json
import os

import pytest

from oracle.cost import amdahl, close_is_faster, expensive_per_step_close, expensive_per_step_original

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cost_model.json")))


def test_cyclooctane_counts():
    c = G["cyclooctane"]
    N = c["references_in_arithmetic"]
    assert expensive_per_step_original(N) == c["original_per_step"]
    close = expensive_per_step_close(N, c["K"])
    assert round(close, 2) == c["close_per_step_printed"]
    assert round(N / c["close_per_step_printed"]) == c["msd_speedup_printed"]


def test_trpcage_counts():
    t = G["trpcage"]
    orig = expensive_per_step_original(t["references"], t["nl_size"], t["nl_stride"])
    assert orig == pytest.approx(t["original_per_step_printed"], abs=1e-12)
    close = expensive_per_step_close(t["references"], t["K"])
    assert round(close, 1) == t["close_per_step_printed"]
    assert round(orig / t["close_per_step_printed"]) == t["msd_speedup_printed"]
    assert close_is_faster(t["references"], t["nl_size"], t["nl_stride"], t["K"])


@pytest.mark.parametrize("name", ["cyclooctane", "trpcage"])
def test_table1_amdahl(name):
    c = G[name]
    S = amdahl(c["table1"]["MSD"], c["msd_speedup_printed"])
    assert round(S, 0 if name == "cyclooctane" else 1) == c["table1"]["S_MSD"]


def test_amdahl_limits():
    assert amdahl(0.9, float("inf")) == pytest.approx(10.0)
    assert amdahl(0.0, 100.0) == 1.0
    assert amdahl(1.0, 8.0) == pytest.approx(8.0)


def test_no_neighbour_list_condition():
    # Without a neighbour list the condition reduces to N > 1 + N/K.
    assert close_is_faster(521, 0, 1, 10000)
    assert not close_is_faster(521, 0, 1, 1)
