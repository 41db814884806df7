"""The identification-rate harness: the GPU's candidates (top-t of the summed scores of each run)
against the oracle's on the same seeded runs, so the reported rates are the oracle's rates."""
import numpy as np
import pytest

from oracle import scores as oscores
from tests.parity import TOL, topk_consistent

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("col_index,runs", [(1, 6), (9, 6), (10, 4)])
def test_identification_rates_match_oracle(gpu_lib, col_index, runs):
    from paper_1409_5000_amd import idrate
    col = idrate.COLUMNS[col_index]
    r = idrate.identification_rates(col, runs, seed=700 + col_index, dtype="f64", workers=4)
    hb = r["batch"]
    ref = oscores.batch_scores(hb, m=0, tol=1e-6, m_max=60, workers=4)
    K = idrate.TARGET_SIZE
    rates_ref = np.empty(runs)
    for g, gsc in enumerate(ref):
        got = r["idx"][g * K:(g + 1) * K]
        ok, _ = topk_consistent(got, gsc.s, K, TOL["f64"])
        assert ok
        cand = oscores.topk(gsc.s, K)
        rates_ref[g] = len(set(cand.tolist()) & set(hb.targets[g].tolist())) / K
    assert np.array_equal(r["rates"], rates_ref)
    assert 0.0 <= r["mean"] <= 1.0 and r["nonfinite"] == 0
