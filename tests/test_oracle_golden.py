"""The oracle still reproduces its reviewed C1 summary (regression fixture
written by tests/golden/make_golden.py from the oracle alone)."""
import json
import os

import pytest

pytestmark = pytest.mark.usefixtures("oracle_lib")

HERE = os.path.dirname(os.path.abspath(__file__))


def test_c1_summary_unchanged():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    with open(os.path.join(HERE, "golden", "c1_oracle_summary.json")) as f:
        want = json.load(f)
    got = mg.summary()
    for k in ("num_pairs", "visible", "keys_sha256", "values_sha256", "n_contrib_sum"):
        assert got[k] == want[k], k
    for k in ("image_sum", "image_max", "final_T_sum"):
        assert got[k] == pytest.approx(want[k], rel=1e-12), k
    assert got["pixel_64_64"] == pytest.approx(want["pixel_64_64"], rel=1e-12)
